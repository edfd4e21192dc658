// Plain schedule: one step = two in-place sweeps over the cell domain.
//   sweep 1: update every H node from the curl of E   (Eq. 2 right column)
//   sweep 2: update every interior E node from the curl of the new H
//            (Eq. 2 left column, J = 0)
// This is the algorithm listing of Sec. 2.1 with the three curl_H (curl_E)
// calls of a half-step merged into one pass; the H boundary needs no work and
// the E boundary (PEC) is the set of nodes sweep 2 never writes.
// Bytes per cell-step (FP32, per-node Ce): sweep 1 reads E, reads and writes
// H (36 B); sweep 2 reads H and Ce, reads and writes E (48 B).
#include "fdtd_internal.h"
#include "yee_update.h"

namespace fdtd {
namespace {

constexpr int kBX = 64, kBY = 4;

template <typename T, bool CH_ARR>
__global__ void __launch_bounds__(kBX *kBY) k_plain_h(Geom g, Fields<T> f, Coefs<T> c)
{
    const int i = blockIdx.x * kBX + threadIdx.x;
    const int j = blockIdx.y * kBY + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= g.nx || j >= g.ny)
        return;
    const long long o = g.at(i, j, k), P = g.plane;
    const int px = g.px;
    const T *ex = f.f[0], *ey = f.f[1], *ez = f.f[2];
    T *hx = f.f[3], *hy = f.f[4], *hz = f.f[5];
    if (i >= 1) {
        T ch = CH_ARR ? c.ch[0][o] : c.ch_s;
        hx[o] = curl_update(hx[o], ch, ey[o + P], ey[o], ez[o + px], ez[o]);
    }
    if (j >= 1) {
        T ch = CH_ARR ? c.ch[1][o] : c.ch_s;
        hy[o] = curl_update(hy[o], ch, ez[o + 1], ez[o], ex[o + P], ex[o]);
    }
    if (k >= 1) {
        T ch = CH_ARR ? c.ch[2][o] : c.ch_s;
        hz[o] = curl_update(hz[o], ch, ex[o + px], ex[o], ey[o + 1], ey[o]);
    }
}

template <typename T, bool CE_ARR>
__global__ void __launch_bounds__(kBX *kBY) k_plain_e(Geom g, Fields<T> f, Coefs<T> c)
{
    const int i = blockIdx.x * kBX + threadIdx.x;
    const int j = blockIdx.y * kBY + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= g.nx || j >= g.ny)
        return;
    const long long o = g.at(i, j, k), P = g.plane;
    const int px = g.px;
    T *ex = f.f[0], *ey = f.f[1], *ez = f.f[2];
    const T *hx = f.f[3], *hy = f.f[4], *hz = f.f[5];
    if (j >= 1 && k >= 1) {
        T ce = CE_ARR ? c.ce[0][o] : c.ce_s;
        ex[o] = curl_update(ex[o], ce, hz[o], hz[o - px], hy[o], hy[o - P]);
    }
    if (i >= 1 && k >= 1) {
        T ce = CE_ARR ? c.ce[1][o] : c.ce_s;
        ey[o] = curl_update(ey[o], ce, hx[o], hx[o - P], hz[o], hz[o - 1]);
    }
    if (i >= 1 && j >= 1) {
        T ce = CE_ARR ? c.ce[2][o] : c.ce_s;
        ez[o] = curl_update(ez[o], ce, hy[o], hy[o - 1], hx[o], hx[o - px]);
    }
}

}  // namespace

template <typename T>
hipError_t launch_plain_step(const Geom &g, const Fields<T> &f, const Coefs<T> &c, hipStream_t s)
{
    dim3 block(kBX, kBY), grid((g.nx + kBX - 1) / kBX, (g.ny + kBY - 1) / kBY, g.nz);
    if (c.ch[0])
        hipLaunchKernelGGL((k_plain_h<T, true>), grid, block, 0, s, g, f, c);
    else
        hipLaunchKernelGGL((k_plain_h<T, false>), grid, block, 0, s, g, f, c);
    if (c.ce[0])
        hipLaunchKernelGGL((k_plain_e<T, true>), grid, block, 0, s, g, f, c);
    else
        hipLaunchKernelGGL((k_plain_e<T, false>), grid, block, 0, s, g, f, c);
    return hipGetLastError();
}

template hipError_t launch_plain_step<float>(const Geom &, const Fields<float> &, const Coefs<float> &,
                                             hipStream_t);
template hipError_t launch_plain_step<double>(const Geom &, const Fields<double> &, const Coefs<double> &,
                                              hipStream_t);

}  // namespace fdtd
