// FP64 diagnostics of a stored state (E^n, H^{n-1/2}), off the timed path.
//
//   W       = sum_E E^2/Ce + sum_H H^{n-1/2} H^{n+1/2} / Ch   (H^{n+1/2} formed
//             here in FP64 from the stored E and H); the leapfrog of Eq. 2
//             conserves it exactly in exact arithmetic because the E curl is
//             minus the transpose of the H curl
//   sum E^2, sum H^2, max |div (H/Ch)| per cell, max |tangential E| on the
//   PEC walls, count of non-finite values.
// A fixed grid of workgroups walks the nodes in a fixed order, so the sums
// do not depend on scheduling.
#include "fdtd_internal.h"
#include "storage.h"

namespace fdtd {
namespace {

constexpr int kBlock = 256;
constexpr int kGrid = 1024;
constexpr int kQ = 6;  // W, sumE2, sumH2, maxdivB, maxEtan, nonfinite

__device__ __forceinline__ bool e_tan(int f, int i, int j, int k, int nx, int ny, int nz)
{
    if (f == 0) return j == 0 || j == ny || k == 0 || k == nz;
    if (f == 1) return i == 0 || i == nx || k == 0 || k == nz;
    return i == 0 || i == nx || j == 0 || j == ny;
}

__device__ __forceinline__ bool h_normal(int f, int i, int j, int k, int nx, int ny, int nz)
{
    if (f == 3) return i == 0 || i == nx;
    if (f == 4) return j == 0 || j == ny;
    return k == 0 || k == nz;
}

template <typename T>
__device__ __forceinline__ double coef_at(const T *arr, T s, bool zero, long long o)
{
    if (zero) return 0.0;
    return arr ? (double)arr[o] : (double)s;
}

template <typename T>
__device__ __forceinline__ double val(const T *a, long long o, long long lo_off)
{
    return (double)get_elem(a, lo_off, o);
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_diag(Geom g, Fields<T> f, Coefs<typename Store<T>::C> c, double *partial)
{
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const long long X = nx + 1, Y = ny + 1, n = X * Y * (nz + 1);
    const long long P = g.plane;
    const int px = g.px;
    double w = 0, se = 0, sh = 0, mdiv = 0, mtan = 0, bad = 0;
    for (long long l = (long long)blockIdx.x * kBlock + threadIdx.x; l < n; l += (long long)kGrid * kBlock) {
        const int i = (int)(l % X);
        const int j = (int)((l / X) % Y);
        const int k = (int)(l / (X * Y));
        const long long o = g.at(i, j, k);
        int ex[6];
        for (int q = 0; q < 6; ++q) {
            int a, b, d;
            extents(g, q, a, b, d);
            ex[q] = i < a && j < b && k < d;
        }
        for (int q = 0; q < 3; ++q) {
            if (!ex[q]) continue;
            double e = val(f.f[q], o, g.lo_rec(q));
            if (!isfinite(e)) bad += 1;
            se += e * e;
            const bool wall = e_tan(q, i, j, k, nx, ny, nz);
            if (wall) {
                mtan = fmax(mtan, fabs(e));
            } else {
                const double ce = coef_at(c.ce[q], c.ce_s, false, o);
                if (ce != 0.0) w += e * e / ce;
            }
        }
        const double Ex0 = ex[0] ? val(f.f[0], o, g.lo_rec(0)) : 0.0, Ey0 = ex[1] ? val(f.f[1], o, g.lo_rec(1)) : 0.0,
                     Ez0 = ex[2] ? val(f.f[2], o, g.lo_rec(2)) : 0.0;
        for (int q = 3; q < 6; ++q) {
            if (!ex[q]) continue;
            double h = val(f.f[q], o, g.lo_rec(q));
            if (!isfinite(h)) bad += 1;
            sh += h * h;
            if (h_normal(q, i, j, k, nx, ny, nz)) continue;
            const double ch = coef_at(c.ch[q - 3], c.ch_s, false, o);
            if (ch == 0.0) continue;
            double d;
            if (q == 3)
                d = (val(f.f[1], o + P, g.lo_rec(1)) - Ey0) - (val(f.f[2], o + px, g.lo_rec(2)) - Ez0);
            else if (q == 4)
                d = (val(f.f[2], o + 1, g.lo_rec(2)) - Ez0) - (val(f.f[0], o + P, g.lo_rec(0)) - Ex0);
            else
                d = (val(f.f[0], o + px, g.lo_rec(0)) - Ex0) - (val(f.f[1], o + 1, g.lo_rec(1)) - Ey0);
            const double hn = h + ch * d;
            w += h * hn / ch;
        }
        if (i < nx && j < ny && k < nz) {
            // B = H/Ch, taken as 0 on wall-normal nodes (constant in time)
            auto b = [&](int q, int ii, int jj, int kk) -> double {
                if (h_normal(q, ii, jj, kk, nx, ny, nz)) return 0.0;
                const long long oo = g.at(ii, jj, kk);
                const double ch = coef_at(c.ch[q - 3], c.ch_s, false, oo);
                return ch != 0.0 ? val(f.f[q], oo, g.lo_rec(q)) / ch : 0.0;
            };
            const double dv = (b(3, i + 1, j, k) - b(3, i, j, k)) + (b(4, i, j + 1, k) - b(4, i, j, k)) +
                              (b(5, i, j, k + 1) - b(5, i, j, k));
            mdiv = fmax(mdiv, fabs(dv));
        }
    }
    __shared__ double red[kQ][kBlock];
    red[0][threadIdx.x] = w;
    red[1][threadIdx.x] = se;
    red[2][threadIdx.x] = sh;
    red[3][threadIdx.x] = mdiv;
    red[4][threadIdx.x] = mtan;
    red[5][threadIdx.x] = bad;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + s];
            red[3][threadIdx.x] = fmax(red[3][threadIdx.x], red[3][threadIdx.x + s]);
            red[4][threadIdx.x] = fmax(red[4][threadIdx.x], red[4][threadIdx.x + s]);
            red[5][threadIdx.x] += red[5][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x < kQ) partial[(long long)blockIdx.x * kQ + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void __launch_bounds__(kBlock) k_diag_final(const double *partial, double *out)
{
    __shared__ double red[kQ][kBlock];
    double acc[kQ] = {0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < kGrid; b += kBlock) {
        for (int q = 0; q < 3; ++q) acc[q] += partial[b * kQ + q];
        acc[3] = fmax(acc[3], partial[b * kQ + 3]);
        acc[4] = fmax(acc[4], partial[b * kQ + 4]);
        acc[5] += partial[b * kQ + 5];
    }
    for (int q = 0; q < kQ; ++q) red[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + s];
            red[3][threadIdx.x] = fmax(red[3][threadIdx.x], red[3][threadIdx.x + s]);
            red[4][threadIdx.x] = fmax(red[4][threadIdx.x], red[4][threadIdx.x + s]);
            red[5][threadIdx.x] += red[5][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x < kQ) out[threadIdx.x] = red[threadIdx.x][0];
}

}  // namespace

size_t diag_partial_doubles() { return (size_t)kGrid * kQ; }

template <typename T>
hipError_t launch_diag(const Geom &g, const Fields<T> &f, const Coefs<typename Store<T>::C> &c, double *partial,
                       double *out_dev, hipStream_t s)
{
    hipLaunchKernelGGL((k_diag<T>), dim3(kGrid), dim3(kBlock), 0, s, g, f, c, partial);
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(kBlock), 0, s, partial, out_dev);
    return hipGetLastError();
}

template hipError_t launch_diag<float>(const Geom &, const Fields<float> &, const Coefs<float> &, double *,
                                       double *, hipStream_t);
template hipError_t launch_diag<double>(const Geom &, const Fields<double> &, const Coefs<double> &, double *,
                                        double *, hipStream_t);
template hipError_t launch_diag<f16>(const Geom &, const Fields<f16> &, const Coefs<float> &, double *, double *,
                                     hipStream_t);
template hipError_t launch_diag<f16c>(const Geom &, const Fields<f16c> &, const Coefs<float> &, double *,
                                      double *, hipStream_t);
template hipError_t launch_diag<bf16c>(const Geom &, const Fields<bf16c> &, const Coefs<float> &, double *,
                                       double *, hipStream_t);
template hipError_t launch_diag<bf16>(const Geom &, const Fields<bf16> &, const Coefs<float> &, double *, double *,
                                      hipStream_t);

}  // namespace fdtd
