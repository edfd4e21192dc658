// Fused schedule: one step = one sweep that marches each x-y tile along z,
// updating H at plane k and then E at plane k before moving to k+1.
//
// This is the GPU form of the paper's sibling fusion of the H curls, the
// boundaries and the E curls into one loop nest (Sec. 3, fusion), done
// out of place: the sweep reads the state from one buffer set and writes the
// next state to the other, so neighbouring workgroups never race (the paper
// updates in place on one CPU thread, Sec. 3, bufferization).
//
// Per plane k, a 64 x TY tile of cells:
//   - E^n at plane k (tile plus the +1 column and +1 row) is staged in LDS;
//     E^n at plane k+1 of the own column is held in registers.
//   - H^{n+1/2} at plane k is computed for the tile; the -1 column and -1 row
//     the E update needs are recomputed by one extra "halo" wave from E^n.
//   - E^{n+1} at plane k follows from H^{n+1/2} at planes k (LDS) and k-1
//     (registers of the previous iteration).
// A z-chunk starts one plane early to rebuild H^{n+1/2} at its first plane-1
// (computed, not stored).
// Bytes per cell-step (FP32): E and H read once and written once (48 B) plus
// the coefficient arrays that are present (12 B for per-node Ce).
#include "fdtd_internal.h"
#include "yee_update.h"

namespace fdtd {
namespace {

constexpr int kTX = 64;

template <typename T, bool CE_ARR, bool CH_ARR, int TY>
__global__ void __launch_bounds__(kTX *(TY + 1))
    k_fused(Geom g, Fields<T> src, Fields<T> dst, Coefs<T> c, int kchunk)
{
    __shared__ T sE[3][TY + 1][kTX + 1];  // E^n plane k at (j0+r, i0+q) -> [r][q]
    __shared__ T sH[3][TY + 1][kTX + 1];  // H^{n+1/2} plane k at (j0+r-1, i0+q-1) -> [r][q]

    const int tx = threadIdx.x, ty = threadIdx.y;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const int i0 = blockIdx.x * kTX, j0 = blockIdx.y * TY;
    const int kb = blockIdx.z * kchunk;
    const int ke = min(nz, kb + kchunk);
    const long long P = g.plane;
    const int px = g.px;
    const bool halo = ty == TY;
    const int i = i0 + tx, j = j0 + ty;
    const bool act = !halo && i < nx && j < ny;

    const T *sEx = src.f[0], *sEy = src.f[1], *sEz = src.f[2];
    const T *sHx = src.f[3], *sHy = src.f[4], *sHz = src.f[5];

    const int kstart = kb > 0 ? kb - 1 : 0;
    T e0 = 0, e1 = 0, e2 = 0;       // E^n at (i, j, k)
    T hpx = 0, hpy = 0;             // H^{n+1/2} at (i, j, k-1)
    if (act) {
        const long long o = g.at(i, j, kstart);
        e0 = sEx[o];
        e1 = sEy[o];
        e2 = sEz[o];
    }

    for (int k = kstart; k < ke; ++k) {
        const bool own = k >= kb;
        // ---------------- loads and E staging ----------------
        T n0 = 0, n1 = 0, n2 = 0, ho0 = 0, ho1 = 0, ho2 = 0;
        T ch0 = c.ch_s, ch1 = c.ch_s, ch2 = c.ch_s, ce0 = c.ce_s, ce1 = c.ce_s, ce2 = c.ce_s;
        long long o = 0;
        // halo-wave registers
        T rEx0 = 0, rEx1 = 0, rEy0 = 0, rEy1 = 0, rEyk = 0, rEz0 = 0, rEz1 = 0, rHz = 0, rHx = 0, rchz = c.ch_s,
          rchx = c.ch_s;
        T cEx0 = 0, cEx1 = 0, cExk = 0, cEy0 = 0, cEy1 = 0, cEz0 = 0, cEz1 = 0, cHz = 0, cHy = 0, cchz = c.ch_s,
          cchy = c.ch_s;
        if (!halo) {
            if (act) {
                o = g.at(i, j, k);
                if (k + 1 < nz) {
                    n0 = sEx[o + P];
                    n1 = sEy[o + P];
                    n2 = sEz[o + P];
                }
                ho0 = sHx[o];
                ho1 = sHy[o];
                ho2 = sHz[o];
                if (CH_ARR) {
                    ch0 = c.ch[0][o];
                    ch1 = c.ch[1][o];
                    ch2 = c.ch[2][o];
                }
                if (CE_ARR && own) {
                    ce0 = c.ce[0][o];
                    ce1 = c.ce[1][o];
                    ce2 = c.ce[2][o];
                }
            }
            sE[0][ty][tx] = e0;
            sE[1][ty][tx] = e1;
            sE[2][ty][tx] = e2;
        } else {
            // +1 row (j0+TY) of Ex, Ez and +1 column (i0+64) of Ey, Ez at plane k
            const int jr = j0 + TY;
            T a = 0, b = 0;
            if (i < nx && jr < ny) {
                const long long q = g.at(i, jr, k);
                a = sEx[q];
                b = sEz[q];
            }
            sE[0][TY][tx] = a;
            sE[1][TY][tx] = 0;
            sE[2][TY][tx] = b;
            if (tx < TY) {
                const int ic = i0 + kTX, jc = j0 + tx;
                T u = 0, v = 0;
                if (ic < nx && jc < ny) {
                    const long long q = g.at(ic, jc, k);
                    u = sEy[q];
                    v = sEz[q];
                }
                sE[0][tx][kTX] = 0;
                sE[1][tx][kTX] = u;
                sE[2][tx][kTX] = v;
            }
            if (own) {
                // -1 row (j0-1): Hz and Hx at (i, j0-1, k)
                const int jh = j0 - 1;
                if (jh >= 0 && i < nx) {
                    const long long q = g.at(i, jh, k);
                    rEx0 = sEx[q];
                    rEx1 = sEx[q + px];
                    rEy0 = sEy[q];
                    rEy1 = (i + 1 < nx) ? sEy[q + 1] : T(0);
                    rEyk = (k + 1 < nz) ? sEy[q + P] : T(0);
                    rEz0 = sEz[q];
                    rEz1 = sEz[q + px];
                    rHz = sHz[q];
                    rHx = sHx[q];
                    if (CH_ARR) {
                        rchz = c.ch[2][q];
                        rchx = c.ch[0][q];
                    }
                }
                // -1 column (i0-1): Hz and Hy at (i0-1, j0+tx, k)
                const int ih = i0 - 1, jc = j0 + tx;
                if (tx < TY && ih >= 0 && jc < ny) {
                    const long long q = g.at(ih, jc, k);
                    cEx0 = sEx[q];
                    cEx1 = (jc + 1 < ny) ? sEx[q + px] : T(0);
                    cExk = (k + 1 < nz) ? sEx[q + P] : T(0);
                    cEy0 = sEy[q];
                    cEy1 = sEy[q + 1];
                    cEz0 = sEz[q];
                    cEz1 = sEz[q + 1];
                    cHz = sHz[q];
                    cHy = sHy[q];
                    if (CH_ARR) {
                        cchz = c.ch[2][q];
                        cchy = c.ch[1][q];
                    }
                }
            }
        }
        __syncthreads();
        // ---------------- H^{n+1/2} at plane k ----------------
        T hx = ho0, hy = ho1, hz = ho2;
        if (!halo) {
            if (act) {
                if (i >= 1)
                    hx = curl_update(ho0, ch0, n1, e1, sE[2][ty + 1][tx], e2);
                if (j >= 1)
                    hy = curl_update(ho1, ch1, sE[2][ty][tx + 1], e2, n0, e0);
                if (k >= 1)
                    hz = curl_update(ho2, ch2, sE[0][ty + 1][tx], e0, sE[1][ty][tx + 1], e1);
                if (own) {
                    T *dHx = dst.f[3], *dHy = dst.f[4], *dHz = dst.f[5];
                    dHx[o] = hx;
                    dHy[o] = hy;
                    dHz[o] = hz;
                }
            }
            sH[0][ty + 1][tx + 1] = hx;
            sH[1][ty + 1][tx + 1] = hy;
            sH[2][ty + 1][tx + 1] = hz;
        } else if (own) {
            // row j0-1: Hz(i, jh) uses Ex(i, jh+1) - Ex(i, jh) and Ey(i+1, jh) - Ey(i, jh);
            //           Hx(i, jh) uses Ey(i, jh, k+1) - Ey(i, jh) and Ez(i, jh+1) - Ez(i, jh)
            T rz = rHz, rx = rHx;
            if (k >= 1)
                rz = curl_update(rHz, rchz, rEx1, rEx0, rEy1, rEy0);
            if (i >= 1)
                rx = curl_update(rHx, rchx, rEyk, rEy0, rEz1, rEz0);
            sH[2][0][tx + 1] = rz;
            sH[0][0][tx + 1] = rx;
            sH[1][0][tx + 1] = 0;
            if (tx < TY) {
                // column i0-1: Hz(ih, jc) uses Ex(ih, jc+1) - Ex(ih, jc) and Ey(i0, jc) - Ey(ih, jc);
                //              Hy(ih, jc) uses Ez(i0, jc) - Ez(ih, jc) and Ex(ih, jc, k+1) - Ex(ih, jc)
                const int jc = j0 + tx;
                T cz = cHz, cy = cHy;
                if (k >= 1)
                    cz = curl_update(cHz, cchz, cEx1, cEx0, cEy1, cEy0);
                if (jc >= 1)
                    cy = curl_update(cHy, cchy, cEz1, cEz0, cExk, cEx0);
                sH[2][tx + 1][0] = cz;
                sH[1][tx + 1][0] = cy;
                sH[0][tx + 1][0] = 0;
            }
        }
        __syncthreads();
        // ---------------- E^{n+1} at plane k ----------------
        if (!halo) {
            if (act && own) {
                T ex = e0, ey = e1, ez = e2;
                if (j >= 1 && k >= 1)
                    ex = curl_update(e0, ce0, hz, sH[2][ty][tx + 1], hy, hpy);
                if (i >= 1 && k >= 1)
                    ey = curl_update(e1, ce1, hx, hpx, hz, sH[2][ty + 1][tx]);
                if (i >= 1 && j >= 1)
                    ez = curl_update(e2, ce2, hy, sH[1][ty + 1][tx], hx, sH[0][ty][tx + 1]);
                T *dEx = dst.f[0], *dEy = dst.f[1], *dEz = dst.f[2];
                dEx[o] = ex;
                dEy[o] = ey;
                dEz[o] = ez;
            }
            hpx = hx;
            hpy = hy;
            e0 = n0;
            e1 = n1;
            e2 = n2;
        }
    }
}

template <typename T, int TY>
hipError_t launch_ty(const Geom &g, const Fields<T> &src, const Fields<T> &dst, const Coefs<T> &c, int zchunk,
                     hipStream_t s)
{
    const int kchunk = (g.nz + zchunk - 1) / zchunk;
    const int nzc = (g.nz + kchunk - 1) / kchunk;
    dim3 block(kTX, TY + 1), grid((g.nx + kTX - 1) / kTX, (g.ny + TY - 1) / TY, nzc);
    const bool cea = c.ce[0] != nullptr, cha = c.ch[0] != nullptr;
    if (cea && cha)
        hipLaunchKernelGGL((k_fused<T, true, true, TY>), grid, block, 0, s, g, src, dst, c, kchunk);
    else if (cea)
        hipLaunchKernelGGL((k_fused<T, true, false, TY>), grid, block, 0, s, g, src, dst, c, kchunk);
    else if (cha)
        hipLaunchKernelGGL((k_fused<T, false, true, TY>), grid, block, 0, s, g, src, dst, c, kchunk);
    else
        hipLaunchKernelGGL((k_fused<T, false, false, TY>), grid, block, 0, s, g, src, dst, c, kchunk);
    return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_fused_step(const Geom &g, const Fields<T> &src, const Fields<T> &dst, const Coefs<T> &c,
                             int zchunk, hipStream_t s)
{
    return launch_ty<T, 8>(g, src, dst, c, zchunk < 1 ? 1 : zchunk, s);
}

template hipError_t launch_fused_step<float>(const Geom &, const Fields<float> &, const Fields<float> &,
                                             const Coefs<float> &, int, hipStream_t);
template hipError_t launch_fused_step<double>(const Geom &, const Fields<double> &, const Fields<double> &,
                                              const Coefs<double> &, int, hipStream_t);

}  // namespace fdtd
