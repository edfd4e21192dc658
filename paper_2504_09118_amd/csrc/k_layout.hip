// Layout conversion and the FP64 coefficient precompute.
//
//   pack    dense staggered array (host layout) -> padded device box, with the
//           PEC boundary (Fig. 1b caption, Sec. 4: tangential E = 0 on walls)
//   unpack  padded device box -> dense staggered array
//   coef    per-node Ce = dt/(dx * eps_edge), Ch = dt/(dx * mu_face) in FP64,
//           rounded once to the storage type (Eq. 2 coefficients dt/eps and
//           dt/mu with the cubic-cell 1/dx folded in)
#include "fdtd_internal.h"
#include "storage.h"

namespace fdtd {
namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ void unflatten(long long l, int X, int Y, int &i, int &j, int &k)
{
    i = (int)(l % X);
    long long r = l / X;
    j = (int)(r % Y);
    k = (int)(r / Y);
}

__device__ __forceinline__ bool e_wall(int field, int i, int j, int k, int nx, int ny, int nz)
{
    switch (field) {
    case 0: return j == 0 || j == ny || k == 0 || k == nz;
    case 1: return i == 0 || i == nx || k == 0 || k == nz;
    case 2: return i == 0 || i == nx || j == 0 || j == ny;
    default: return false;
    }
}

// Wall-normal H node: its update reads only wall-tangential E, so it never changes.
__device__ __forceinline__ bool h_wall_normal(int field, int i, int j, int k, int nx, int ny, int nz)
{
    switch (field) {
    case 3: return i == 0 || i == nx;
    case 4: return j == 0 || j == ny;
    case 5: return k == 0 || k == nz;
    default: return false;
    }
}

template <typename S, typename T>
__global__ void __launch_bounds__(kBlock) k_pack(Geom g, int field, int X, int Y, long long n,
                                                 const S *__restrict__ src, T *dst, T *dst2, double scale)
{
    long long l = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (l >= n)
        return;
    int i, j, k;
    unflatten(l, X, Y, i, j, k);
    // scaled in FP64 (exact for scale 1); 16-bit storage: rounded to FP32, then to the 16-bit type
    typename Store<T>::C v = to_compute<T>((double)src[l] * scale);
    if (e_wall(field, i, j, k, g.nx, g.ny, g.nz))
        v = 0;
    // a wall-normal H of -0 is stored as +0 (equal values): sweeps that add the zero curl to
    // every H node then keep every bit
    if (h_wall_normal(field, i, j, k, g.nx, g.ny, g.nz) && v == 0)
        v = 0;
    long long o = g.at(i, j, k);
    put_elem(dst, g.lo_rec(field), o, v);
    if (dst2)
        put_elem(dst2, g.lo_rec(field), o, v);
}

template <typename T, typename S>
__global__ void __launch_bounds__(kBlock) k_unpack(Geom g, int field, int X, int Y, long long n,
                                                   const T *__restrict__ src, S *__restrict__ dst, double scale)
{
    long long l = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (l >= n)
        return;
    int i, j, k;
    unflatten(l, X, Y, i, j, k);
    dst[l] = (S)((double)get_elem(src, g.lo_rec(field), g.at(i, j, k)) / scale);
}

__device__ __forceinline__ double mat(const double *m, int nx, int ny, int i, int j, int k)
{
    return m ? m[(long long)i + (long long)nx * ((long long)j + (long long)ny * k)] : 1.0;
}

// One thread per node of component `field` (0..2 E edges, 3..5 H faces).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_coef(Geom g, int field, int X, int Y, long long n, double dx,
                                                 double dt, const double *__restrict__ m, T *out, double fac)
{
    long long l = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (l >= n)
        return;
    int i, j, k;
    unflatten(l, X, Y, i, j, k);
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    double c = 0.0;
    switch (field) {
    case 0:  // x-edge: cells (i, j-1..j, k-1..k)
        if (j > 0 && j < ny && k > 0 && k < nz) {
            double a = (mat(m, nx, ny, i, j - 1, k - 1) + mat(m, nx, ny, i, j, k - 1)) +
                       (mat(m, nx, ny, i, j - 1, k) + mat(m, nx, ny, i, j, k));
            c = dt / (dx * (a * 0.25));
        }
        break;
    case 1:  // y-edge: cells (i-1..i, j, k-1..k)
        if (i > 0 && i < nx && k > 0 && k < nz) {
            double a = (mat(m, nx, ny, i - 1, j, k - 1) + mat(m, nx, ny, i - 1, j, k)) +
                       (mat(m, nx, ny, i, j, k - 1) + mat(m, nx, ny, i, j, k));
            c = dt / (dx * (a * 0.25));
        }
        break;
    case 2:  // z-edge: cells (i-1..i, j-1..j, k)
        if (i > 0 && i < nx && j > 0 && j < ny) {
            double a = (mat(m, nx, ny, i - 1, j - 1, k) + mat(m, nx, ny, i, j - 1, k)) +
                       (mat(m, nx, ny, i - 1, j, k) + mat(m, nx, ny, i, j, k));
            c = dt / (dx * (a * 0.25));
        }
        break;
    case 3:  // x-face between cells (i-1, j, k) and (i, j, k)
        if (i > 0 && i < nx)
            c = dt / (dx * ((mat(m, nx, ny, i - 1, j, k) + mat(m, nx, ny, i, j, k)) * 0.5));
        break;
    case 4:
        if (j > 0 && j < ny)
            c = dt / (dx * ((mat(m, nx, ny, i, j - 1, k) + mat(m, nx, ny, i, j, k)) * 0.5));
        break;
    default:
        if (k > 0 && k < nz)
            c = dt / (dx * ((mat(m, nx, ny, i, j, k - 1) + mat(m, nx, ny, i, j, k)) * 0.5));
        break;
    }
    out[g.at(i, j, k)] = (T)(c * fac);  // exact for fac 1; one rounding, to nearest even
}

inline unsigned blocks_for(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

template <typename S, typename T>
hipError_t launch_pack(const Geom &g, int field, const S *src, T *dst, T *dst2, hipStream_t s, double scale)
{
    int X, Y, Z;
    extents(g, field, X, Y, Z);
    long long n = (long long)X * Y * Z;
    hipLaunchKernelGGL((k_pack<S, T>), dim3(blocks_for(n)), dim3(kBlock), 0, s, g, field, X, Y, n, src, dst,
                       dst2, scale);
    return hipGetLastError();
}

template <typename T, typename S>
hipError_t launch_unpack(const Geom &g, int field, const T *src, S *dst, hipStream_t s, double scale)
{
    int X, Y, Z;
    extents(g, field, X, Y, Z);
    long long n = (long long)X * Y * Z;
    hipLaunchKernelGGL((k_unpack<T, S>), dim3(blocks_for(n)), dim3(kBlock), 0, s, g, field, X, Y, n, src, dst,
                       scale);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_coef(const Geom &g, double dx, double dt, const double *eps, const double *mu, T *ce[3],
                       T *ch[3], hipStream_t s, const double *fac)
{
    for (int f = 0; f < 6; ++f) {
        T *out = f < 3 ? ce[f] : ch[f - 3];
        if (!out)
            continue;
        int X, Y, Z;
        extents(g, f, X, Y, Z);
        long long n = (long long)X * Y * Z;
        hipLaunchKernelGGL((k_coef<T>), dim3(blocks_for(n)), dim3(kBlock), 0, s, g, f, X, Y, n, dx, dt,
                           f < 3 ? eps : mu, out, fac ? fac[f] : 1.0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

template hipError_t launch_pack<float, float>(const Geom &, int, const float *, float *, float *, hipStream_t, double);
template hipError_t launch_pack<double, float>(const Geom &, int, const double *, float *, float *, hipStream_t, double);
template hipError_t launch_pack<float, double>(const Geom &, int, const float *, double *, double *, hipStream_t, double);
template hipError_t launch_pack<double, double>(const Geom &, int, const double *, double *, double *,
                                                hipStream_t, double);
template hipError_t launch_pack<float, f16>(const Geom &, int, const float *, f16 *, f16 *, hipStream_t, double);
template hipError_t launch_pack<double, f16>(const Geom &, int, const double *, f16 *, f16 *, hipStream_t, double);
template hipError_t launch_pack<float, bf16>(const Geom &, int, const float *, bf16 *, bf16 *, hipStream_t, double);
template hipError_t launch_pack<double, bf16>(const Geom &, int, const double *, bf16 *, bf16 *, hipStream_t, double);
template hipError_t launch_pack<float, f16c>(const Geom &, int, const float *, f16c *, f16c *, hipStream_t, double);
template hipError_t launch_pack<double, f16c>(const Geom &, int, const double *, f16c *, f16c *, hipStream_t, double);
template hipError_t launch_pack<float, bf16c>(const Geom &, int, const float *, bf16c *, bf16c *, hipStream_t,
                                              double);
template hipError_t launch_pack<double, bf16c>(const Geom &, int, const double *, bf16c *, bf16c *, hipStream_t,
                                               double);
template hipError_t launch_unpack<f16c, float>(const Geom &, int, const f16c *, float *, hipStream_t, double);
template hipError_t launch_unpack<f16c, double>(const Geom &, int, const f16c *, double *, hipStream_t, double);
template hipError_t launch_unpack<bf16c, float>(const Geom &, int, const bf16c *, float *, hipStream_t, double);
template hipError_t launch_unpack<bf16c, double>(const Geom &, int, const bf16c *, double *, hipStream_t, double);
template hipError_t launch_unpack<f16, float>(const Geom &, int, const f16 *, float *, hipStream_t, double);
template hipError_t launch_unpack<f16, double>(const Geom &, int, const f16 *, double *, hipStream_t, double);
template hipError_t launch_unpack<bf16, float>(const Geom &, int, const bf16 *, float *, hipStream_t, double);
template hipError_t launch_unpack<bf16, double>(const Geom &, int, const bf16 *, double *, hipStream_t, double);
template hipError_t launch_unpack<float, float>(const Geom &, int, const float *, float *, hipStream_t, double);
template hipError_t launch_unpack<float, double>(const Geom &, int, const float *, double *, hipStream_t, double);
template hipError_t launch_unpack<double, float>(const Geom &, int, const double *, float *, hipStream_t, double);
template hipError_t launch_unpack<double, double>(const Geom &, int, const double *, double *, hipStream_t, double);
template hipError_t launch_coef<float>(const Geom &, double, double, const double *, const double *, float *[3],
                                       float *[3], hipStream_t, const double *);
template hipError_t launch_coef<double>(const Geom &, double, double, const double *, const double *,
                                        double *[3], double *[3], hipStream_t, const double *);

}  // namespace fdtd
