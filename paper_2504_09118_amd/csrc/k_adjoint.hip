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
#include <cstdlib>

#include "fdtd_internal.h"
#include "yee_update.h"

// Every product below is rounded on its own: no multiply is fused into a neighbouring add or
// subtract, so the fused reverse sweep and the one-cell-per-thread kernels evaluate the same
// rounding sequence and give the same bits (the curl updates are explicit fused multiply-adds).
#pragma clang fp contract(off)

namespace fdtd {
namespace {

constexpr int kBX = 64, kBY = 4;

// A product rounded on its own (contraction is off in this file).
__device__ __forceinline__ float rmul(float a, float b) { return a * b; }
__device__ __forceinline__ double rmul(double a, double b) { return a * b; }

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

// J = sum over the rows 1..N of (sum over the probes of E^2), each row summed in probe order and
// added to J in row order: the bits of the per-step accumulation. The recorded values are read
// into LDS by the whole workgroup, a chunk at a time, and summed by one thread.
constexpr int kSumChunk = 4096;
__global__ void __launch_bounds__(kProbeBlock) k_probe_objective(const double *__restrict__ rec, long long nrows,
                                                                 int np, double *J)
{
    __shared__ double buf[kSumChunk];
    const int t = threadIdx.x;
    const long long total = nrows * (long long)np;  // values of rows 1..N (row 0 is not part of J)
    const int rows_per = kSumChunk / np;
    double acc_j = 0.0;
    for (long long row0 = 0; row0 < nrows; row0 += rows_per) {
        const long long nr = nrows - row0 < rows_per ? nrows - row0 : rows_per;
        const long long base = (row0 + 1) * (long long)np, cnt = nr * np;
        for (long long q = t; q < cnt; q += kProbeBlock) buf[q] = rec[base + q];
        __syncthreads();
        if (t == 0) {
            for (long long r = 0; r < nr; ++r) {
                double acc = 0.0;
                for (int p = 0; p < np; ++p) {
                    const double v = buf[r * np + p];
                    acc += rmul(v, v);
                }
                acc_j += acc;
            }
        }
        __syncthreads();
    }
    (void)total;
    if (t == 0)
        *J = acc_j;
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
        mx[o] = curl_update(mx[o], m1, rmul(cy[o + P], ly[o + P]), rmul(cy[o], ly[o]), rmul(cz[o + px], lz[o + px]),
                            rmul(cz[o], lz[o]));
    if (j >= 1)
        my[o] = curl_update(my[o], m1, rmul(cz[o + 1], lz[o + 1]), rmul(cz[o], lz[o]), rmul(cx[o + P], lx[o + P]),
                            rmul(cx[o], lx[o]));
    if (k >= 1)
        mz[o] = curl_update(mz[o], m1, rmul(cx[o + px], lx[o + px]), rmul(cx[o], lx[o]), rmul(cy[o + 1], ly[o + 1]),
                            rmul(cy[o], ly[o]));
}

// gCe += lam (L H^{n+1/2}); lam -= L (Ch mu), on the interior E nodes.
// GM 0: gCe in g (FP64) directly; 1: into the FP32 group sums p; 2: into p, then
// p is added to g and cleared (the last step of a group).
template <int GM, typename T>
__device__ __forceinline__ void add_gce(double *g, float *p, long long o, T l, T lh)
{
    if constexpr (GM == 0) {
        (void)p;
        g[o] += rmul((double)l, (double)lh);
    } else {
        const float v = p[o] + rmul((float)l, (float)lh);
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
    auto b = [&](int q, const T *m, long long idx) -> T { return rmul(CH_ARR ? c.ch[q][idx] : c.ch_s, m[idx]); };
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

// ---------------------------------------------------------------------------
// Fused reverse step: one z-marching sweep, laid out like the forward slab
// sweep (k_slab.hip): a workgroup of R waves owns an x-y tile 64V cells wide
// and R-2 rows high and marches a z-chunk; wave 0 (row j0-1) only rebuilds mu'
// for the first own row's lam update, wave R-1 (row j0+R-2) only stages Ce lam
// for the last own row's mu update, lane 0 carries the -1 column and lane 63
// the +1 column. Per plane k:
//   stage Ce lam and h = H^{n+1/2} of plane k in LDS;
//   mu'  = mu - K(Ce lam)                 (the H-update stencil, coefficient -1)
//   stage Ch mu' of plane k in LDS;
//   gCe += lam (L h), lam' = lam - L(Ch mu')  (the E-update stencil)
//   lam' += 2 E^n at the probes of plane k (probe order, as a serial loop)
// reading (lam, mu) from src and writing (lam', mu') to dst (a neighbour tile's
// halo must see the old values); the gCe sums are updated in place (one owner
// per node). The products Ce lam and Ch mu' are rounded in T, then
// differenced, with the operands of k_adj_mu / k_adj_lam: the same bits.
// GM as for k_adj_lam. The x-neighbour operands at the tile edge come from LDS.
template <typename T, int V>
struct AVec {
    typedef T type __attribute__((ext_vector_type(V)));
};

#define FDTD_GLOBAL __attribute__((address_space(1)))

__device__ __forceinline__ FDTD_GLOBAL char *auni(const void *p)
{
    const unsigned long long v = (unsigned long long)p;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return (FDTD_GLOBAL char *)(((unsigned long long)hi << 32) | lo);
}

template <typename T, int V>
__device__ __forceinline__ typename AVec<T, V>::type ald(const T *plane, unsigned boff)
{
    return *(FDTD_GLOBAL const typename AVec<T, V>::type *)(auni(plane) + boff);
}

template <typename T>
__device__ __forceinline__ T ald1(const T *plane, unsigned boff)
{
    return *(FDTD_GLOBAL const T *)(auni(plane) + boff);
}

template <typename T, int V>
__device__ __forceinline__ void ast(T *plane, unsigned boff, const typename AVec<T, V>::type &x)
{
    *(FDTD_GLOBAL typename AVec<T, V>::type *)(auni(plane) + boff) = x;
}


template <typename T, int V, int R, bool CH_ARR, int GM>
__global__ void __launch_bounds__(64 * R)
    k_adj_slab(Geom g, Fields<T> src, Fields<T> dst, Coefs<T> c, const T *__restrict__ hxp, const T *__restrict__ hyp,
               const T *__restrict__ hzp, double *gxp, double *gyp, double *gzp, float *pxp, float *pyp, float *pzp,
               ProbeList pl, const double *rec_row, int kchunk, int ntx, int nty, int ntiles, int xcd_remap)
{
    using vec = typename AVec<T, V>::type;
    using fvec = typename AVec<float, V>::type;
    constexpr int TX = 64 * V;
    constexpr int LP = TX + 2 * V;
    constexpr int HO = V;  // column of the first own cell in the H-like arrays; HO-1 is the -1 column
    constexpr int kX = 8;
    __shared__ __attribute__((aligned(16))) T sE[3][R][LP];   // Ce lam, plane k; column TX: +1 column
    __shared__ __attribute__((aligned(16))) T sB[3][R][LP];   // Ch mu', plane k; column HO-1: -1 column
    __shared__ __attribute__((aligned(16))) T sHh[3][R][LP];  // h = H^{n+1/2}, plane k; column HO-1: -1 column
    __shared__ T sExm[R];                                      // (Ce lam)_x at (i0-1, j0-1+r, k)

    const int nper = (ntiles + kX - 1) / kX;
    const int b = blockIdx.x;
    const int t = xcd_remap ? (b % kX) * nper + b / kX : b;
    if (t >= ntiles)
        return;
    const int tile_x = t % ntx;
    const int tile_y = (t / ntx) % nty;
    const int zc = t / (ntx * nty);

    const int tx = threadIdx.x, r = threadIdx.y;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const int i0 = tile_x * TX;
    const int j0 = tile_y * (R - 2);
    const int j = j0 - 1 + r;
    const int kb = zc * kchunk;
    const int ke = min(nz, kb + kchunk);
    const long long P = g.plane;
    const int px = g.px;
    const int ib = i0 + tx * V;
    const bool rowok = j >= 0 && j < ny;
    const bool act = rowok && ib < nx;
    const bool hrow = r < R - 1;            // computes mu'
    const bool erow = r >= 1 && r < R - 1;  // owns its row: lam update, gCe, stores
    const bool xl = tx == 0 && rowok && i0 >= 1;
    const bool xr = tx == 63 && rowok && i0 + TX < nx;
    const unsigned xoff = (unsigned)((tx == 0 ? i0 - 1 : i0 + TX) + px * j) * (unsigned)sizeof(T);
    const unsigned off = (unsigned)(ib + px * j) * (unsigned)sizeof(T);
    const unsigned offp = (unsigned)(ib + px * j) * (unsigned)sizeof(float);
    const unsigned lin = (unsigned)(ib + px * j);  // in-plane element offset of the lane's first cell

    const int kstart = kb > 0 ? kb - 1 : 0;
    const vec zero = (vec)(T)0;
    const T m1 = (T)-1;
    const T *Lx = src.f[0], *Ly = src.f[1], *Lz = src.f[2];
    const T *Mx = src.f[3], *My = src.f[4], *Mz = src.f[5];

    // lam at k (l) and k+1 (n), Ce at k and k+1, old mu at k, h at k and (x, y) at k-1,
    // (Ch mu')_(x, y) at k-1, the FP32 gCe sums at k, Ch at k
    vec l0 = zero, l1 = zero, l2 = zero, n0 = zero, n1 = zero, n2 = zero;
    vec ce0 = zero, ce1 = zero, ce2 = zero, nc0 = zero, nc1 = zero, nc2 = zero;
    vec mo0 = zero, mo1 = zero, mo2 = zero;
    vec h0 = zero, h1 = zero, h2 = zero, hpx = zero, hpy = zero, bpx = zero, bpy = zero;
    const fvec fzero = (fvec)0.0f;
    fvec gp0 = fzero, gp1 = fzero, gp2 = fzero;
    vec ch0 = (vec)c.ch_s, ch1 = (vec)c.ch_s, ch2 = (vec)c.ch_s;
    // -1 column (lane 0): lam_x, Ce_x at k and k+1, lam_y Ce_y, lam_z Ce_z, old mu_z, mu_y, Ch z, y,
    // h_z, h_y; +1 column (lane 63): lam_y Ce_y, lam_z Ce_z
    T xlx0 = 0, xlx1 = 0, xcx0 = 0, xcx1 = 0, xly = 0, xcy = 0, xlz = 0, xcz = 0, xmz = 0, xmy = 0;
    T xchz = c.ch_s, xchy = c.ch_s, xhz = 0, xhy = 0;
    {
        const long long pk = (long long)kstart * P;
        if (act) {
            l0 = ald<T, V>(Lx + pk, off);
            l1 = ald<T, V>(Ly + pk, off);
            l2 = ald<T, V>(Lz + pk, off);
            ce0 = ald<T, V>(c.ce[0] + pk, off);
            ce1 = ald<T, V>(c.ce[1] + pk, off);
            ce2 = ald<T, V>(c.ce[2] + pk, off);
            if (kstart + 1 < nz) {
                n0 = ald<T, V>(Lx + pk + P, off);
                n1 = ald<T, V>(Ly + pk + P, off);
                n2 = ald<T, V>(Lz + pk + P, off);
                nc0 = ald<T, V>(c.ce[0] + pk + P, off);
                nc1 = ald<T, V>(c.ce[1] + pk + P, off);
                nc2 = ald<T, V>(c.ce[2] + pk + P, off);
            }
            if (hrow) {
                mo0 = ald<T, V>(Mx + pk, off);
                mo1 = ald<T, V>(My + pk, off);
                mo2 = ald<T, V>(Mz + pk, off);
                if (CH_ARR) {
                    ch0 = ald<T, V>(c.ch[0] + pk, off);
                    ch1 = ald<T, V>(c.ch[1] + pk, off);
                    ch2 = ald<T, V>(c.ch[2] + pk, off);
                }
            }
            h0 = ald<T, V>(hxp + pk, off);
            h1 = ald<T, V>(hyp + pk, off);
            h2 = ald<T, V>(hzp + pk, off);
            if (GM != 0 && erow) {
                gp0 = ald<float, V>(pxp + pk, offp);
                gp1 = ald<float, V>(pyp + pk, offp);
                gp2 = ald<float, V>(pzp + pk, offp);
            }
        }
        if (xl) {
            xlx0 = ald1(Lx + pk, xoff);
            xcx0 = ald1(c.ce[0] + pk, xoff);
            if (kstart + 1 < nz) {
                xlx1 = ald1(Lx + pk + P, xoff);
                xcx1 = ald1(c.ce[0] + pk + P, xoff);
            }
            xly = ald1(Ly + pk, xoff);
            xcy = ald1(c.ce[1] + pk, xoff);
            xlz = ald1(Lz + pk, xoff);
            xcz = ald1(c.ce[2] + pk, xoff);
            xmz = ald1(Mz + pk, xoff);
            xmy = ald1(My + pk, xoff);
            if (CH_ARR) {
                xchz = ald1(c.ch[2] + pk, xoff);
                xchy = ald1(c.ch[1] + pk, xoff);
            }
            xhz = ald1(hzp + pk, xoff);
            xhy = ald1(hyp + pk, xoff);
        }
        if (xr) {
            xly = ald1(Ly + pk, xoff);
            xcy = ald1(c.ce[1] + pk, xoff);
            xlz = ald1(Lz + pk, xoff);
            xcz = ald1(c.ce[2] + pk, xoff);
        }
    }
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0) before the loop (see the forward sweeps)

    for (int k = kstart; k < ke; ++k) {
        const bool own = k >= kb;
        const bool more = k + 1 < ke;
        const long long pk = (long long)k * P;
        // ---------------- prefetch: lam, Ce at k+2; mu, h, gCe sums, Ch at k+1 ----------------
        vec p0 = zero, p1 = zero, p2 = zero, pc0 = zero, pc1 = zero, pc2 = zero;
        vec q0 = zero, q1 = zero, q2 = zero, ph0 = zero, ph1 = zero, ph2 = zero;
        fvec pg0 = fzero, pg1 = fzero, pg2 = fzero;
        vec pch0 = (vec)c.ch_s, pch1 = (vec)c.ch_s, pch2 = (vec)c.ch_s;
        T pxlx = 0, pxcx = 0, pxly = 0, pxcy = 0, pxlz = 0, pxcz = 0, pxmz = 0, pxmy = 0;
        T pxchz = c.ch_s, pxchy = c.ch_s, pxhz = 0, pxhy = 0;
        if (more) {
            const long long p1k = pk + P;
            if (act) {
                if (k + 2 < nz) {
                    p0 = ald<T, V>(Lx + p1k + P, off);
                    p1 = ald<T, V>(Ly + p1k + P, off);
                    p2 = ald<T, V>(Lz + p1k + P, off);
                    pc0 = ald<T, V>(c.ce[0] + p1k + P, off);
                    pc1 = ald<T, V>(c.ce[1] + p1k + P, off);
                    pc2 = ald<T, V>(c.ce[2] + p1k + P, off);
                }
                if (hrow) {
                    q0 = ald<T, V>(Mx + p1k, off);
                    q1 = ald<T, V>(My + p1k, off);
                    q2 = ald<T, V>(Mz + p1k, off);
                    if (CH_ARR) {
                        pch0 = ald<T, V>(c.ch[0] + p1k, off);
                        pch1 = ald<T, V>(c.ch[1] + p1k, off);
                        pch2 = ald<T, V>(c.ch[2] + p1k, off);
                    }
                }
                ph0 = ald<T, V>(hxp + p1k, off);
                ph1 = ald<T, V>(hyp + p1k, off);
                ph2 = ald<T, V>(hzp + p1k, off);
                if (GM != 0 && erow) {
                    pg0 = ald<float, V>(pxp + p1k, offp);
                    pg1 = ald<float, V>(pyp + p1k, offp);
                    pg2 = ald<float, V>(pzp + p1k, offp);
                }
            }
            if (xl) {
                if (k + 2 < nz) {
                    pxlx = ald1(Lx + p1k + P, xoff);
                    pxcx = ald1(c.ce[0] + p1k + P, xoff);
                }
                pxly = ald1(Ly + p1k, xoff);
                pxcy = ald1(c.ce[1] + p1k, xoff);
                pxlz = ald1(Lz + p1k, xoff);
                pxcz = ald1(c.ce[2] + p1k, xoff);
                pxmz = ald1(Mz + p1k, xoff);
                pxmy = ald1(My + p1k, xoff);
                if (CH_ARR) {
                    pxchz = ald1(c.ch[2] + p1k, xoff);
                    pxchy = ald1(c.ch[1] + p1k, xoff);
                }
                pxhz = ald1(hzp + p1k, xoff);
                pxhy = ald1(hyp + p1k, xoff);
            }
            if (xr) {
                pxly = ald1(Ly + p1k, xoff);
                pxcy = ald1(c.ce[1] + p1k, xoff);
                pxlz = ald1(Lz + p1k, xoff);
                pxcz = ald1(c.ce[2] + p1k, xoff);
            }
        }
        // ---------------- stage Ce lam and h of plane k ----------------
        vec cl0, cl1, cl2;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            cl0[v] = rmul(ce0[v], l0[v]);
            cl1[v] = rmul(ce1[v], l1[v]);
            cl2[v] = rmul(ce2[v], l2[v]);
        }
        *(vec *)&sE[0][r][tx * V] = cl0;
        *(vec *)&sE[1][r][tx * V] = cl1;
        *(vec *)&sE[2][r][tx * V] = cl2;
        *(vec *)&sHh[0][r][HO + tx * V] = h0;
        *(vec *)&sHh[1][r][HO + tx * V] = h1;
        *(vec *)&sHh[2][r][HO + tx * V] = h2;
        if (tx == 0) {
            sExm[r] = rmul(xcx0, xlx0);
            sHh[2][r][HO - 1] = xhz;
            sHh[1][r][HO - 1] = xhy;
            sHh[0][r][HO - 1] = 0;
        }
        if (tx == 63) {
            sE[1][r][TX] = rmul(xcy, xly);  // 0 unless lane 63 staged a real +1 column
            sE[2][r][TX] = rmul(xcz, xlz);
        }
        __syncthreads();
        // ---------------- mu' at plane k ----------------
        vec mx = mo0, my = mo1, mz = mo2;
        vec bx, by, bz;
        if (hrow) {
            if (act) {
                const vec czj = *(const vec *)&sE[2][r + 1][tx * V];  // (Ce lam)_z (i, j+1)
                const vec cxj = *(const vec *)&sE[0][r + 1][tx * V];  // (Ce lam)_x (i, j+1)
                const T czr = sE[2][r][tx * V + V];                    // (Ce lam)_z (ib+V, j)
                const T cyr = sE[1][r][tx * V + V];                    // (Ce lam)_y (ib+V, j)
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const int i = ib + v;
                    if (i >= nx)
                        continue;  // a cell past the domain keeps its loaded value
                    const T cz_ip = v + 1 < V ? cl2[v + 1] : czr;
                    const T cy_ip = v + 1 < V ? cl1[v + 1] : cyr;
                    if (i >= 1)
                        mx[v] = curl_update(mo0[v], m1, rmul(nc1[v], n1[v]), cl1[v], czj[v], cl2[v]);
                    if (j >= 1)
                        my[v] = curl_update(mo1[v], m1, cz_ip, cl2[v], rmul(nc0[v], n0[v]), cl0[v]);
                    if (k >= 1)
                        mz[v] = curl_update(mo2[v], m1, cxj[v], cl0[v], cy_ip, cl1[v]);
                }
            }
#pragma unroll
            for (int v = 0; v < V; ++v) {
                bx[v] = rmul(ch0[v], mx[v]);
                by[v] = rmul(ch1[v], my[v]);
                bz[v] = rmul(ch2[v], mz[v]);
            }
            *(vec *)&sB[0][r][HO + tx * V] = bx;
            *(vec *)&sB[1][r][HO + tx * V] = by;
            *(vec *)&sB[2][r][HO + tx * V] = bz;
            if (tx == 0) {
                // -1 column: mu'_z(i0-1, j) and mu'_y(i0-1, j), the operands of k_adj_mu
                T cz = xmz, cy = xmy;
                if (xl) {
                    const T cxu = sExm[r + 1];  // (Ce lam)_x (i0-1, j+1); 0 beyond the domain
                    if (k >= 1)
                        cz = curl_update(xmz, m1, cxu, rmul(xcx0, xlx0), cl1[0], rmul(xcy, xly));
                    if (j >= 1)
                        cy = curl_update(xmy, m1, cl2[0], rmul(xcz, xlz), rmul(xcx1, xlx1), rmul(xcx0, xlx0));
                }
                sB[2][r][HO - 1] = rmul(xchz, cz);
                sB[1][r][HO - 1] = rmul(xchy, cy);
                sB[0][r][HO - 1] = 0;
            }
        }
        else {
            bx = zero;
            by = zero;
            bz = zero;
        }
        if (hrow && erow && act && own) {
            ast<T, V>(dst.f[3] + pk, off, mx);
            ast<T, V>(dst.f[4] + pk, off, my);
            ast<T, V>(dst.f[5] + pk, off, mz);
        }
        __syncthreads();
        // ---------------- gCe and lam' at plane k ----------------
        vec lx = l0, ly = l1, lz = l2;
        if (erow && act && own) {
            const vec bzj = *(const vec *)&sB[2][r - 1][HO + tx * V];   // (Ch mu')_z (i, j-1)
            const vec bxj = *(const vec *)&sB[0][r - 1][HO + tx * V];   // (Ch mu')_x (i, j-1)
            const T bzl = sB[2][r][HO + tx * V - 1];                    // (Ch mu')_z (ib-1, j)
            const T byl = sB[1][r][HO + tx * V - 1];                    // (Ch mu')_y (ib-1, j)
            const vec hzj = *(const vec *)&sHh[2][r - 1][HO + tx * V];  // h_z (i, j-1)
            const vec hxj = *(const vec *)&sHh[0][r - 1][HO + tx * V];  // h_x (i, j-1)
            const T hzl = sHh[2][r][HO + tx * V - 1];                   // h_z (ib-1, j)
            const T hyl = sHh[1][r][HO + tx * V - 1];                   // h_y (ib-1, j)
            const long long o0 = pk + (long long)lin;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int i = ib + v;
                if (i >= nx)
                    continue;
                const long long o = o0 + v;
                const T bz_im = v > 0 ? bz[v - 1] : bzl;
                const T by_im = v > 0 ? by[v - 1] : byl;
                const T hz_im = v > 0 ? h2[v - 1] : hzl;
                const T hy_im = v > 0 ? h1[v - 1] : hyl;
                if (j >= 1 && k >= 1) {
                    const T lh = (h2[v] - hzj[v]) - (h1[v] - hpy[v]);
                    if constexpr (GM == 0) {
                        gxp[o] += rmul((double)l0[v], (double)lh);
                    } else {
                        gp0[v] = gp0[v] + rmul((float)l0[v], (float)lh);
                        if constexpr (GM == 2) {
                            gxp[o] += (double)gp0[v];
                            gp0[v] = 0.0f;
                        }
                    }
                    lx[v] = curl_update(l0[v], m1, bz[v], bzj[v], by[v], bpy[v]);
                }
                if (i >= 1 && k >= 1) {
                    const T lh = (h0[v] - hpx[v]) - (h2[v] - hz_im);
                    if constexpr (GM == 0) {
                        gyp[o] += rmul((double)l1[v], (double)lh);
                    } else {
                        gp1[v] = gp1[v] + rmul((float)l1[v], (float)lh);
                        if constexpr (GM == 2) {
                            gyp[o] += (double)gp1[v];
                            gp1[v] = 0.0f;
                        }
                    }
                    ly[v] = curl_update(l1[v], m1, bx[v], bpx[v], bz[v], bz_im);
                }
                if (i >= 1 && j >= 1) {
                    const T lh = (h1[v] - hy_im) - (h0[v] - hxj[v]);
                    if constexpr (GM == 0) {
                        gzp[o] += rmul((double)l2[v], (double)lh);
                    } else {
                        gp2[v] = gp2[v] + rmul((float)l2[v], (float)lh);
                        if constexpr (GM == 2) {
                            gzp[o] += (double)gp2[v];
                            gp2[v] = 0.0f;
                        }
                    }
                    lz[v] = curl_update(l2[v], m1, by[v], by_im, bx[v], bxj[v]);
                }
            }
        }
        // probe terms of this plane, in probe order (duplicates add in turn); the plane tests are
        // uniform, only the lane that owns a probe node adds
        if (rec_row) {
            const bool mine = erow && act && own;
            for (int q = 0; q < pl.np; ++q) {
                if (pl.pk[q] != k)
                    continue;
                const int d = pl.pxy[q] - (int)lin;
                const T add = (T)(2.0 * rec_row[q]);
                const int f = pl.pf[q];
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    if (!mine || d != v)
                        continue;
                    if (f == 0)
                        lx[v] = lx[v] + add;
                    else if (f == 1)
                        ly[v] = ly[v] + add;
                    else
                        lz[v] = lz[v] + add;
                }
            }
        }
        if (erow && act && own) {
            ast<T, V>(dst.f[0] + pk, off, lx);
            ast<T, V>(dst.f[1] + pk, off, ly);
            ast<T, V>(dst.f[2] + pk, off, lz);
            if (GM != 0) {
                ast<float, V>(pxp + pk, offp, gp0);
                ast<float, V>(pyp + pk, offp, gp1);
                ast<float, V>(pzp + pk, offp, gp2);
            }
        }
        // ---------------- rotate ----------------
        hpx = h0;
        hpy = h1;
        bpx = bx;
        bpy = by;
        l0 = n0;
        l1 = n1;
        l2 = n2;
        n0 = p0;
        n1 = p1;
        n2 = p2;
        ce0 = nc0;
        ce1 = nc1;
        ce2 = nc2;
        nc0 = pc0;
        nc1 = pc1;
        nc2 = pc2;
        mo0 = q0;
        mo1 = q1;
        mo2 = q2;
        h0 = ph0;
        h1 = ph1;
        h2 = ph2;
        gp0 = pg0;
        gp1 = pg1;
        gp2 = pg2;
        if (CH_ARR) {
            ch0 = pch0;
            ch1 = pch1;
            ch2 = pch2;
            xchz = pxchz;
            xchy = pxchy;
        }
        xlx0 = xlx1;
        xcx0 = xcx1;
        xlx1 = pxlx;
        xcx1 = pxcx;
        xly = pxly;
        xcy = pxcy;
        xlz = pxlz;
        xcz = pxcz;
        xmz = pxmz;
        xmy = pxmy;
        xhz = pxhz;
        xhy = pxhy;
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

hipError_t launch_probe_objective(const double *rec, long long nrows, int np, double *J, hipStream_t s)
{
    if (np <= 0 || np > kSumChunk)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_probe_objective, dim3(1), dim3(kProbeBlock), 0, s, rec, nrows, np, J);
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

namespace {

template <typename T, int V, int R>
hipError_t launch_adj_slab_cfg(const Geom &g, const Fields<T> &src, const Fields<T> &dst, const Coefs<T> &c,
                               const T *const hist[3], double *const gce[3], float *const gpart[3], bool close_group,
                               const ProbeList &pl, const double *rec_row, int zchunk, hipStream_t s)
{
    constexpr int TX = 64 * V;
    const int kchunk = (g.nz + zchunk - 1) / zchunk;
    const int nzc = (g.nz + kchunk - 1) / kchunk;
    const int ntx = (g.nx + TX - 1) / TX, nty = (g.ny + R - 3) / (R - 2);
    const int ntiles = ntx * nty * nzc;
    const int nblocks = (ntiles + 7) / 8 * 8;
    dim3 block(64, R), grid(nblocks);
    float *p0 = gpart ? gpart[0] : nullptr, *p1 = gpart ? gpart[1] : nullptr, *p2 = gpart ? gpart[2] : nullptr;
    const int gm = !gpart ? 0 : (close_group ? 2 : 1);
    const bool cha = c.ch[0] != nullptr;
    const int rm = xcd_remap() ? 1 : 0;
#define FDTD_ADJ_SLAB(CHV, GMV)                                                                                     \
    hipLaunchKernelGGL((k_adj_slab<T, V, R, CHV, GMV>), grid, block, 0, s, g, src, dst, c, hist[0], hist[1],     \
                       hist[2], gce[0], gce[1], gce[2], p0, p1, p2, pl, rec_row, kchunk, ntx, nty, ntiles, rm)
    if (gm == 0) {
        if (cha) FDTD_ADJ_SLAB(true, 0);
        else FDTD_ADJ_SLAB(false, 0);
    } else if (gm == 1) {
        if (cha) FDTD_ADJ_SLAB(true, 1);
        else FDTD_ADJ_SLAB(false, 1);
    } else {
        if (cha) FDTD_ADJ_SLAB(true, 2);
        else FDTD_ADJ_SLAB(false, 2);
    }
#undef FDTD_ADJ_SLAB
    return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_adj_sweep(const Geom &g, const Fields<T> &src, const Fields<T> &dst, const Coefs<T> &c,
                            const T *const hist[3], double *const gce[3], float *const gpart[3], bool close_group,
                            const ProbeList &pl, const double *rec_row, int zchunk, hipStream_t s)
{
    zchunk = zchunk < 1 ? 1 : zchunk;
    const double *rr = pl.np > 0 ? rec_row : nullptr;
    // tile shape (FDTD_ADJ_VARIANT): 1, the default, 2 cells per lane and 8 waves (128 x 6 own
    // cells; measured fastest at 128^3: backward 38 ms against 43 ms with 1 cell per lane and
    // 16 waves, 0); 2: 2 cells and 16 waves; 3: 1 cell and 8 waves
    static const int variant = [] {
        const char *e = getenv("FDTD_ADJ_VARIANT");
        return (e && *e) ? atoi(e) : 1;
    }();
    static const int zc_env = [] {
        const char *e = getenv("FDTD_ADJ_ZCHUNKS");
        return (e && *e) ? atoi(e) : 0;
    }();
    if (zc_env > 0)
        zchunk = zc_env;
    if constexpr (sizeof(T) == 8)
        return launch_adj_slab_cfg<T, 1, 8>(g, src, dst, c, hist, gce, gpart, close_group, pl, rr, zchunk, s);
    else {
        if (variant == 0)
            return launch_adj_slab_cfg<T, 1, 16>(g, src, dst, c, hist, gce, gpart, close_group, pl, rr, zchunk, s);
        if (variant == 2)
            return launch_adj_slab_cfg<T, 2, 16>(g, src, dst, c, hist, gce, gpart, close_group, pl, rr, zchunk, s);
        if (variant == 3)
            return launch_adj_slab_cfg<T, 1, 8>(g, src, dst, c, hist, gce, gpart, close_group, pl, rr, zchunk, s);
        return launch_adj_slab_cfg<T, 2, 8>(g, src, dst, c, hist, gce, gpart, close_group, pl, rr, zchunk, s);
    }
}

#define FDTD_ADJ_INST(T)                                                                                        \
    template hipError_t launch_source_probe<T>(const Fields<T> &, int, long long, double, int, const int *,   \
                                               const long long *, double *, double *, hipStream_t);            \
    template hipError_t launch_adj_probe<T>(const Fields<T> &, int, const int *, const long long *,           \
                                            const double *, hipStream_t);                                      \
    template hipError_t launch_adj_step<T>(const Geom &, const Fields<T> &, const Coefs<T> &, const T *const[3], \
                                           double *const[3], float *const[3], bool, hipStream_t);              \
    template hipError_t launch_grad_eps<T>(const Geom &, const Coefs<T> &, double *const[3], double, double *, \
                                           hipStream_t);                                                       \
    template hipError_t launch_adj_sweep<T>(const Geom &, const Fields<T> &, const Fields<T> &, const Coefs<T> &, \
                                            const T *const[3], double *const[3], float *const[3], bool,           \
                                            const ProbeList &, const double *, int, hipStream_t);
FDTD_ADJ_INST(float)
FDTD_ADJ_INST(double)
#undef FDTD_ADJ_INST

}  // namespace fdtd
