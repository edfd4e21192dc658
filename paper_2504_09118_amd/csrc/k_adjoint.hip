// Reverse-time (adjoint) sweeps of the driven leapfrog, and the point source /
// probe kernel of its forward pass.
//
// Forward (Sec. 2 Eq. 2 with Ampere's current density kept as a point source
// added to one E node after each E update):
//   H^{n+1/2} = H^{n-1/2} + Ch (K E^n),  E^{n+1} = E^n + Ce (L H^{n+1/2}) + w_{n+1}
//   J = sum_{n=1..N} sum_p (E^n at probe p)^2
// Reverse step n (n = N-1 .. 0), with lam = dJ/dE, mu = dJ/dH:
//   mu  -= K (Ce lam)                  adjoint of the E update's H dependence
//   gCe += lam (L H^{n+1/2})           before lam changes (lam^{n+1})
//   lam -= L (Ch mu)                   adjoint of the H update's E dependence
//   lam += 2 E^n at the probes         (n >= 1)
// K and L are the curl stencils of the forward sweeps; the Yee curls satisfy
// L = -K^T on the updated nodes, which turns the transposes into the same
// stencils with the coefficient inside the curl and a minus sign. Nodes the
// forward never updates (wall-tangential E, wall-normal H) keep lam = mu = 0.
// The gradient accumulates in FP64; the stencils run in the storage type. With
// FP32 storage each step's gCe term is first summed in FP32 over fixed groups
// of kAdjGroup reverse steps (the steps n with n % kAdjGroup == 0 close a
// group, whatever the checkpoint interval, so the bits do not depend on it)
// and each group's sum is added to the FP64 total: the FP64 array is read and
// written once per group instead of every step.
#include "fdtd_internal.h"
#include "yee_update.h"

namespace fdtd {
namespace {

constexpr int kBX = 64, kBY = 4;

constexpr int kProbeBlock = 256;

// Point source and probe reads of one driven step, one workgroup: thread 0 adds w to the
// source node; probe p is read by thread p (mod the block) in parallel, a probe on the source
// node adding w itself with the same rounding as the stored value (the source store may land
// later); thread 0 then sums the squares in probe order, so J has the bits of a serial loop.
template <typename T>
__global__ void __launch_bounds__(kProbeBlock) k_source_probe(Fields<T> f, int sf, long long so, double w, int np,
                                                              const int *__restrict__ pf,
                                                              const long long *__restrict__ po, double *rec_row,
                                                              double *J)
{
    const int t = threadIdx.x;
    if (rec_row) {
        for (int p = t; p < np; p += kProbeBlock) {
            T v = f.f[pf[p]][po[p]];
            if (pf[p] == sf && po[p] == so)
                v = v + (T)w;
            rec_row[p] = (double)v;
        }
    }
    __syncthreads();
    if (t != 0)
        return;
    if (sf >= 0)
        f.f[sf][so] = f.f[sf][so] + (T)w;
    if (!rec_row)
        return;
    double acc = 0.0;
    for (int p = 0; p < np; ++p) {
        const double v = rec_row[p];
        acc += v * v;
    }
    *J += acc;
}

// lam += 2 E^n at the probes. Thread p handles probe p (mod the block) unless an earlier
// probe names the same node; the first one adds the contributions of all its duplicates in
// probe order, as a serial loop would.
template <typename T>
__global__ void __launch_bounds__(kProbeBlock) k_adj_probe(Fields<T> lam, int np, const int *__restrict__ pf,
                                                           const long long *__restrict__ po,
                                                           const double *__restrict__ rec_row)
{
    for (int p = threadIdx.x; p < np; p += kProbeBlock) {
        const int fp = pf[p];
        const long long op = po[p];
        bool first = true;
        for (int q = 0; q < p && first; ++q)
            first = !(pf[q] == fp && po[q] == op);
        if (!first)
            continue;
        T v = lam.f[fp][op];
        for (int q = p; q < np; ++q)
            if (pf[q] == fp && po[q] == op)
                v = v + (T)(2.0 * rec_row[q]);
        lam.f[fp][op] = v;
    }
}

// mu -= K (Ce lam) on the H nodes the forward H sweep updates.
template <typename T>
__global__ void __launch_bounds__(kBX *kBY) k_adj_mu(Geom g, Fields<T> a, Coefs<T> c)
{
    const int i = blockIdx.x * kBX + threadIdx.x;
    const int j = blockIdx.y * kBY + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= g.nx || j >= g.ny)
        return;
    const long long o = g.at(i, j, k), P = g.plane;
    const int px = g.px;
    const T *lx = a.f[0], *ly = a.f[1], *lz = a.f[2];
    T *mx = a.f[3], *my = a.f[4], *mz = a.f[5];
    const T *cx = c.ce[0], *cy = c.ce[1], *cz = c.ce[2];
    const T m1 = (T)-1;
    if (i >= 1)
        mx[o] = curl_update(mx[o], m1, cy[o + P] * ly[o + P], cy[o] * ly[o], cz[o + px] * lz[o + px], cz[o] * lz[o]);
    if (j >= 1)
        my[o] = curl_update(my[o], m1, cz[o + 1] * lz[o + 1], cz[o] * lz[o], cx[o + P] * lx[o + P], cx[o] * lx[o]);
    if (k >= 1)
        mz[o] = curl_update(mz[o], m1, cx[o + px] * lx[o + px], cx[o] * lx[o], cy[o + 1] * ly[o + 1], cy[o] * ly[o]);
}

// gCe += lam (L H^{n+1/2}); lam -= L (Ch mu), on the interior E nodes.
// GM 0: gCe in g (FP64) directly; 1: into the FP32 group sums p; 2: into p, then
// p is added to g and cleared (the last step of a group).
template <int GM, typename T>
__device__ __forceinline__ void add_gce(double *g, float *p, long long o, T l, T lh)
{
    if constexpr (GM == 0) {
        (void)p;
        g[o] += (double)l * (double)lh;
    } else {
        const float v = p[o] + (float)l * (float)lh;
        if constexpr (GM == 2) {
            g[o] += (double)v;
            p[o] = 0.0f;
        } else {
            (void)g;
            p[o] = v;
        }
    }
}

template <typename T, bool CH_ARR, int GM>
__global__ void __launch_bounds__(kBX *kBY)
    k_adj_lam(Geom g, Fields<T> a, Coefs<T> c, const T *__restrict__ hx, const T *__restrict__ hy,
              const T *__restrict__ hz, double *gx, double *gy, double *gz, float *px, float *py, float *pz)
{
    const int i = blockIdx.x * kBX + threadIdx.x;
    const int j = blockIdx.y * kBY + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= g.nx || j >= g.ny)
        return;
    const long long o = g.at(i, j, k), P = g.plane;
    const int px_ = g.px;
    T *lx = a.f[0], *ly = a.f[1], *lz = a.f[2];
    const T *mx = a.f[3], *my = a.f[4], *mz = a.f[5];
    auto b = [&](int q, const T *m, long long idx) -> T { return (CH_ARR ? c.ch[q][idx] : c.ch_s) * m[idx]; };
    const T m1 = (T)-1;
    if (j >= 1 && k >= 1) {
        const T l = lx[o];
        const T lh = (hz[o] - hz[o - px_]) - (hy[o] - hy[o - P]);
        add_gce<GM>(gx, px, o, l, lh);
        lx[o] = curl_update(l, m1, b(2, mz, o), b(2, mz, o - px_), b(1, my, o), b(1, my, o - P));
    }
    if (i >= 1 && k >= 1) {
        const T l = ly[o];
        const T lh = (hx[o] - hx[o - P]) - (hz[o] - hz[o - 1]);
        add_gce<GM>(gy, py, o, l, lh);
        ly[o] = curl_update(l, m1, b(0, mx, o), b(0, mx, o - P), b(2, mz, o), b(2, mz, o - 1));
    }
    if (i >= 1 && j >= 1) {
        const T l = lz[o];
        const T lh = (hy[o] - hy[o - 1]) - (hx[o] - hx[o - px_]);
        add_gce<GM>(gz, pz, o, l, lh);
        lz[o] = curl_update(l, m1, b(1, my, o), b(1, my, o - 1), b(0, mx, o), b(0, mx, o - px_));
    }
}

// dJ/d eps per cell: the twelve edges of the cell, dCe/d eps_cell = -Ce^2 dx / dt / 4
// (Ce = dt / (dx mean eps), mean over the edge's four cells). FP64.
template <typename T>
__global__ void __launch_bounds__(256) k_grad_eps(Geom g, Coefs<T> c, const double *__restrict__ gx,
                                                  const double *__restrict__ gy, const double *__restrict__ gz,
                                                  double dx_over_dt, double *__restrict__ out)
{
    const long long n = (long long)g.nx * g.ny * g.nz;
    const long long l = (long long)blockIdx.x * 256 + threadIdx.x;
    if (l >= n)
        return;
    const int i = (int)(l % g.nx);
    const int j = (int)((l / g.nx) % g.ny);
    const int k = (int)(l / ((long long)g.nx * g.ny));
    auto w = [&](int q, const double *gq, int ii, int jj, int kk) {
        const long long o = g.at(ii, jj, kk);
        const double cv = (double)c.ce[q][o];
        return gq[o] * cv * cv;
    };
    const double sx = (w(0, gx, i, j, k) + w(0, gx, i, j + 1, k)) + (w(0, gx, i, j, k + 1) + w(0, gx, i, j + 1, k + 1));
    const double sy = (w(1, gy, i, j, k) + w(1, gy, i + 1, j, k)) + (w(1, gy, i, j, k + 1) + w(1, gy, i + 1, j, k + 1));
    const double sz = (w(2, gz, i, j, k) + w(2, gz, i + 1, j, k)) + (w(2, gz, i, j + 1, k) + w(2, gz, i + 1, j + 1, k));
    out[l] = -0.25 * dx_over_dt * ((sx + sy) + sz);
}

}  // namespace

template <typename T>
hipError_t launch_source_probe(const Fields<T> &f, int sf, long long so, double w, int np, const int *pf,
                               const long long *po, double *rec_row, double *J, hipStream_t s)
{
    hipLaunchKernelGGL((k_source_probe<T>), dim3(1), dim3(kProbeBlock), 0, s, f, sf, so, w, np, pf, po, rec_row, J);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_probe(const Fields<T> &lam, int np, const int *pf, const long long *po, const double *rec_row,
                            hipStream_t s)
{
    hipLaunchKernelGGL((k_adj_probe<T>), dim3(1), dim3(kProbeBlock), 0, s, lam, np, pf, po, rec_row);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_step(const Geom &g, const Fields<T> &a, const Coefs<T> &c, const T *const hist[3],
                           double *const gce[3], float *const gpart[3], bool close_group, hipStream_t s)
{
    dim3 block(kBX, kBY), grid((g.nx + kBX - 1) / kBX, (g.ny + kBY - 1) / kBY, g.nz);
    hipLaunchKernelGGL((k_adj_mu<T>), grid, block, 0, s, g, a, c);
    float *p0 = gpart ? gpart[0] : nullptr, *p1 = gpart ? gpart[1] : nullptr, *p2 = gpart ? gpart[2] : nullptr;
#define FDTD_ADJ_LAM(CHV, GMV)                                                                                   \
    hipLaunchKernelGGL((k_adj_lam<T, CHV, GMV>), grid, block, 0, s, g, a, c, hist[0], hist[1], hist[2], gce[0], \
                       gce[1], gce[2], p0, p1, p2)
    const int gm = !gpart ? 0 : (close_group ? 2 : 1);
    const bool cha = c.ch[0] != nullptr;
    if (gm == 0) {
        if (cha) FDTD_ADJ_LAM(true, 0);
        else FDTD_ADJ_LAM(false, 0);
    } else if (gm == 1) {
        if (cha) FDTD_ADJ_LAM(true, 1);
        else FDTD_ADJ_LAM(false, 1);
    } else {
        if (cha) FDTD_ADJ_LAM(true, 2);
        else FDTD_ADJ_LAM(false, 2);
    }
#undef FDTD_ADJ_LAM
    return hipGetLastError();
}

template <typename T>
hipError_t launch_grad_eps(const Geom &g, const Coefs<T> &c, double *const gce[3], double dx_over_dt, double *out,
                           hipStream_t s)
{
    const long long n = (long long)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL((k_grad_eps<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, c, gce[0], gce[1],
                       gce[2], dx_over_dt, out);
    return hipGetLastError();
}

#define FDTD_ADJ_INST(T)                                                                                        \
    template hipError_t launch_source_probe<T>(const Fields<T> &, int, long long, double, int, const int *,   \
                                               const long long *, double *, double *, hipStream_t);            \
    template hipError_t launch_adj_probe<T>(const Fields<T> &, int, const int *, const long long *,           \
                                            const double *, hipStream_t);                                      \
    template hipError_t launch_adj_step<T>(const Geom &, const Fields<T> &, const Coefs<T> &, const T *const[3], \
                                           double *const[3], float *const[3], bool, hipStream_t);              \
    template hipError_t launch_grad_eps<T>(const Geom &, const Coefs<T> &, double *const[3], double, double *, \
                                           hipStream_t);
FDTD_ADJ_INST(float)
FDTD_ADJ_INST(double)
#undef FDTD_ADJ_INST

}  // namespace fdtd
