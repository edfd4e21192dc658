// Slab schedule: the fused z-marching sweep (see k_fused.hip) tuned for
// gfx950 HBM bandwidth.
//
// A workgroup is R waves; wave r owns cell row j = j0 - 1 + r of a tile that
// is 64V cells wide in x, and marches it along z:
//   - wave 0 (row j0-1) only rebuilds H^{n+1/2}, which the first own row's
//     E update needs; wave R-1 (row j0+R-2) only stages E^n, which the last
//     own row's H update needs; waves 1..R-2 own their rows. All waves run
//     the same code (the role only masks loads, math and stores), so the
//     halo costs no extra registers;
//   - each lane owns V consecutive x-cells and moves them with one V-wide
//     access per component (dwordx2 for V = 2 FP32);
//   - lane 0 also carries the -1 column (rebuilds H at i0-1) and lane 63 the
//     +1 column (stages E at i0+64V), through the same pipeline;
//   - the global loads for plane k+1 (E at k+2, old H, coefficients at k+1)
//     are issued at the top of plane k, so a full plane of work hides them;
//   - plane-k E and H are exchanged through LDS between waves and lanes;
//   - the per-plane base of every array is wave-uniform (scalar registers)
//     and lanes add 32-bit offsets;
//   - workgroups are numbered so that the hardware's round-robin placement
//     over the 8 XCDs gives each XCD one contiguous block of tiles: halo
//     re-reads of neighbouring tiles then hit the same 4 MB L2.
// Arithmetic per node is curl_update with the same operands as every other
// schedule, so the results are bit-identical.
#include "fdtd_internal.h"
#include "yee_update.h"

namespace fdtd {
namespace {

constexpr int kXcds = 8;

template <typename T, int V>
struct VecOf {
    typedef T type __attribute__((ext_vector_type(V)));
};
template <typename T>
struct VecOf<T, 1> {
    typedef T type;
};

template <typename T, int V>
__device__ __forceinline__ T el(const typename VecOf<T, V>::type &x, int v)
{
    if constexpr (V == 1) {
        return x;
    } else {
        return x[v];
    }
}

template <typename T, int V>
__device__ __forceinline__ void set_el(typename VecOf<T, V>::type &x, int v, T val)
{
    if constexpr (V == 1) {
        x = val;
    } else {
        x[v] = val;
    }
}

// A plane base pointer is the same for every lane; pinning it to scalar
// registers (and to the global address space) lets each access be
// "scalar base + 32-bit lane offset".
#define FDTD_GLOBAL __attribute__((address_space(1)))

__device__ __forceinline__ FDTD_GLOBAL char *uni(const void *p)
{
    const unsigned long long v = (unsigned long long)p;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return (FDTD_GLOBAL char *)(((unsigned long long)hi << 32) | lo);
}

// plane: wave-uniform base of one z-plane; boff: per-lane byte offset inside it
template <typename T, int V>
__device__ __forceinline__ typename VecOf<T, V>::type ld(const T *plane, unsigned boff)
{
    return *(FDTD_GLOBAL const typename VecOf<T, V>::type *)(uni(plane) + boff);
}

template <typename T>
__device__ __forceinline__ T ld1(const T *plane, unsigned boff)
{
    return *(FDTD_GLOBAL const T *)(uni(plane) + boff);
}

template <typename T, int V>
__device__ __forceinline__ void st(T *plane, unsigned boff, const typename VecOf<T, V>::type &x)
{
    *(FDTD_GLOBAL typename VecOf<T, V>::type *)(uni(plane) + boff) = x;
}

template <typename T>
__device__ __forceinline__ void st1(T *plane, unsigned boff, T x)
{
    *(FDTD_GLOBAL T *)(uni(plane) + boff) = x;
}

// Buffer store of a lane's V cells to a plane: raw buffer with the plane as its
// range, so an offset at or beyond plane_bytes is dropped by the hardware range
// check. Every lane issues the store every plane (lanes that must not write pass
// kDrop), which keeps the number of memory operations after the prefetch loads
// the same on every path; the wait for the prefetch then never covers stores.
constexpr unsigned kDrop = 0x80000000u;
constexpr int kRawBufferWord3 = 0x00020000;  // gfx9 raw buffer: 32-bit data format, no swizzle
// cache policy of the stores: non-temporal (the written state is not read again in this
// sweep), so written lines leave L2 early and the lines of the tiles' shared halos stay
constexpr int kStoreNT = 2;

template <typename T, int V, bool NT>
__device__ __forceinline__ void st_plane(T *plane, unsigned plane_bytes, unsigned boff,
                                         const typename VecOf<T, V>::type &x)
{
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(plane, 0, (int)plane_bytes, kRawBufferWord3);
    constexpr int bytes = (int)sizeof(T) * V;
    if constexpr (bytes == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, boff, 0, NT ? kStoreNT : 0);
    } else if constexpr (bytes == 8) {
        typedef unsigned u2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, x), r, boff, 0, NT ? kStoreNT : 0);
    } else {
        typedef unsigned u4 __attribute__((ext_vector_type(4)));
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, x), r, boff, 0, NT ? kStoreNT : 0);
    }
}

template <typename T, int V, int R, bool CE_ARR, bool CH_ARR, bool NT>
__global__ void __launch_bounds__(64 * R)
    k_slab(Geom g, Fields<T> src, Fields<T> dst, Coefs<T> c, int kchunk, int ntx, int nty, int ntiles,
               int xcd_remap, SlabExtras xt)
{
    using vec = typename VecOf<T, V>::type;
    constexpr int TX = 64 * V;       // tile width (cells)
    constexpr int LP = TX + 2 * V;   // LDS row pitch (elements), keeps V-wide accesses aligned
    constexpr int HO = V;            // column of the first own cell in sH; the -1 column is HO-1
    __shared__ __attribute__((aligned(16))) T sE[3][R][LP];  // E^n plane k: [r][q] <-> (j0-1+r, i0+q); q = TX is +1 col
    __shared__ __attribute__((aligned(16))) T sH[3][R][LP];  // H^{n+1/2} plane k: [r][HO+q] <-> (j0-1+r, i0+q)
    __shared__ T sExm[R];                                     // Ex^n at (i0-1, j0-1+r, k)

    // XCD-aware tile numbering: hardware block b runs on XCD b % 8.
    const int nper = (ntiles + kXcds - 1) / kXcds;
    const int b = blockIdx.x;
    const int t = xcd_remap ? (b % kXcds) * nper + b / kXcds : b;
    if (t >= ntiles)
        return;  // the whole workgroup leaves before any barrier
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
    const bool act = rowok && ib < nx;            // lane has cells in the domain
    const bool hrow = r < R - 1;                  // computes H (all but the E-provider row)
    const bool erow = r >= 1 && r < R - 1;        // owns its row: E update and stores
    // x-halo lanes: lane 0 rebuilds H at i0-1, lane 63 stages E at i0+TX
    const bool xl = tx == 0 && rowok && i0 >= 1;
    const bool xr = tx == 63 && rowok && i0 + TX < nx;
    // in-plane byte offsets (32-bit, so the plane base stays in scalar registers)
    const unsigned xoff = (unsigned)((tx == 0 ? i0 - 1 : i0 + TX) + px * j) * (unsigned)sizeof(T);  // halo column
    const unsigned off = (unsigned)(ib + px * j) * (unsigned)sizeof(T);                               // lane's cells

    const int kstart = kb > 0 ? kb - 1 : 0;
    const vec zero = (vec)(T)0;
    const T *Ex = src.f[0], *Ey = src.f[1], *Ez = src.f[2];
    const T *Hx = src.f[3], *Hy = src.f[4], *Hz = src.f[5];

    // pipeline registers: E^n at k (e) and k+1 (n), old H (ho) and coefficients at k
    vec e0 = zero, e1 = zero, e2 = zero, n0 = zero, n1 = zero, n2 = zero;
    vec ho0 = zero, ho1 = zero, ho2 = zero;
    vec ce0 = (vec)c.ce_s, ce1 = (vec)c.ce_s, ce2 = (vec)c.ce_s;
    vec ch0 = (vec)c.ch_s, ch1 = (vec)c.ch_s, ch2 = (vec)c.ch_s;
    vec hpx = zero, hpy = zero;  // H^{n+1/2} at k-1
    // halo column: lane 0 holds Ex (k, k+1), Ey, Ez, old Hz, Hy, Ch at (i0-1, j);
    // lane 63 holds Ey, Ez at (i0+TX, j)
    T xa0 = 0, xa1 = 0, xb = 0, xc = 0, xd = 0, xe = 0, xchz = c.ch_s, xchy = c.ch_s;
    {
        const long long pk = (long long)kstart * P;
        if (act) {
            e0 = ld<T, V>(Ex + pk, off);
            e1 = ld<T, V>(Ey + pk, off);
            e2 = ld<T, V>(Ez + pk, off);
            if (kstart + 1 < nz) {
                n0 = ld<T, V>(Ex + pk + P, off);
                n1 = ld<T, V>(Ey + pk + P, off);
                n2 = ld<T, V>(Ez + pk + P, off);
            }
            if (hrow) {
                ho0 = ld<T, V>(Hx + pk, off);
                ho1 = ld<T, V>(Hy + pk, off);
                ho2 = ld<T, V>(Hz + pk, off);
                if (CH_ARR) {
                    ch0 = ld<T, V>(c.ch[0] + pk, off);
                    ch1 = ld<T, V>(c.ch[1] + pk, off);
                    ch2 = ld<T, V>(c.ch[2] + pk, off);
                }
            }
            if (CE_ARR && erow) {
                ce0 = ld<T, V>(c.ce[0] + pk, off);
                ce1 = ld<T, V>(c.ce[1] + pk, off);
                ce2 = ld<T, V>(c.ce[2] + pk, off);
            }
        }
        if (xl) {
            xa0 = ld1(Ex + pk, xoff);
            if (kstart + 1 < nz)
                xa1 = ld1(Ex + pk + P, xoff);
            xb = ld1(Ey + pk, xoff);
            xc = ld1(Ez + pk, xoff);
            xd = ld1(Hz + pk, xoff);
            xe = ld1(Hy + pk, xoff);
            if (CH_ARR) {
                xchz = ld1(c.ch[2] + pk, xoff);
                xchy = ld1(c.ch[1] + pk, xoff);
            }
        }
        if (xr) {
            xb = ld1(Ey + pk, xoff);
            xc = ld1(Ez + pk, xoff);
        }
    }

    // vmcnt(0): the prologue loads land in registers the loop carries; without this wait the
    // compiler's conservative merge at the loop head makes every plane wait for its own prefetch
    __builtin_amdgcn_s_waitcnt(0x0F70);
    const unsigned plane_bytes = (unsigned)(P * (long long)sizeof(T));

    for (int k = kstart; k < ke; ++k) {
        const bool own = k >= kb;
        const bool more = k + 1 < ke;
        const long long pk = (long long)k * P;
        // ---------------- prefetch plane k+1 ----------------
        vec p0 = zero, p1 = zero, p2 = zero, q0 = zero, q1 = zero, q2 = zero;
        vec pce0 = (vec)c.ce_s, pce1 = (vec)c.ce_s, pce2 = (vec)c.ce_s;
        vec pch0 = (vec)c.ch_s, pch1 = (vec)c.ch_s, pch2 = (vec)c.ch_s;
        T pxa = 0, pxb = 0, pxc = 0, pxd = 0, pxe = 0, pxchz = c.ch_s, pxchy = c.ch_s;
        if (more) {
            const long long p1k = pk + P;
            if (act) {
                if (k + 2 < nz) {
                    p0 = ld<T, V>(Ex + p1k + P, off);
                    p1 = ld<T, V>(Ey + p1k + P, off);
                    p2 = ld<T, V>(Ez + p1k + P, off);
                }
                if (hrow) {
                    q0 = ld<T, V>(Hx + p1k, off);
                    q1 = ld<T, V>(Hy + p1k, off);
                    q2 = ld<T, V>(Hz + p1k, off);
                    if (CH_ARR) {
                        pch0 = ld<T, V>(c.ch[0] + p1k, off);
                        pch1 = ld<T, V>(c.ch[1] + p1k, off);
                        pch2 = ld<T, V>(c.ch[2] + p1k, off);
                    }
                }
                if (CE_ARR && erow) {
                    pce0 = ld<T, V>(c.ce[0] + p1k, off);
                    pce1 = ld<T, V>(c.ce[1] + p1k, off);
                    pce2 = ld<T, V>(c.ce[2] + p1k, off);
                }
            }
            if (xl) {
                if (k + 2 < nz)
                    pxa = ld1(Ex + p1k + P, xoff);
                pxb = ld1(Ey + p1k, xoff);
                pxc = ld1(Ez + p1k, xoff);
                pxd = ld1(Hz + p1k, xoff);
                pxe = ld1(Hy + p1k, xoff);
                if (CH_ARR) {
                    pxchz = ld1(c.ch[2] + p1k, xoff);
                    pxchy = ld1(c.ch[1] + p1k, xoff);
                }
            }
            if (xr) {
                pxb = ld1(Ey + p1k, xoff);
                pxc = ld1(Ez + p1k, xoff);
            }
        }
        // ---------------- stage E^n of plane k ----------------
        *(vec *)&sE[0][r][tx * V] = e0;
        *(vec *)&sE[1][r][tx * V] = e1;
        *(vec *)&sE[2][r][tx * V] = e2;
        if (tx == 0)
            sExm[r] = xa0;
        if (tx == 63) {
            sE[1][r][TX] = xb;  // 0 unless lane 63 staged a real +1 column
            sE[2][r][TX] = xc;
        }
        __syncthreads();
        // ---------------- H^{n+1/2} at plane k ----------------
        vec hx = ho0, hy = ho1, hz = ho2;
        if (hrow) {
            if (act) {
                const vec ezj = *(const vec *)&sE[2][r + 1][tx * V];  // Ez(i, j+1)
                const vec exj = *(const vec *)&sE[0][r + 1][tx * V];  // Ex(i, j+1)
                const T ezr = sE[2][r][tx * V + V];                    // Ez(ib+V, j)
                const T eyr = sE[1][r][tx * V + V];                    // Ey(ib+V, j)
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const int i = ib + v;
                    if (i >= nx)
                        continue;  // a cell past the domain keeps its loaded (constant) value
                    const T ez_ip = v + 1 < V ? el<T, V>(e2, v + 1) : ezr;
                    const T ey_ip = v + 1 < V ? el<T, V>(e1, v + 1) : eyr;
                    if (i >= 1)
                        set_el<T, V>(hx, v, curl_update(el<T, V>(ho0, v), el<T, V>(ch0, v), el<T, V>(n1, v),
                                                        el<T, V>(e1, v), el<T, V>(ezj, v), el<T, V>(e2, v)));
                    if (j >= 1)
                        set_el<T, V>(hy, v, curl_update(el<T, V>(ho1, v), el<T, V>(ch1, v), ez_ip, el<T, V>(e2, v),
                                                        el<T, V>(n0, v), el<T, V>(e0, v)));
                    if (k >= 1)
                        set_el<T, V>(hz, v, curl_update(el<T, V>(ho2, v), el<T, V>(ch2, v), el<T, V>(exj, v),
                                                        el<T, V>(e0, v), ey_ip, el<T, V>(e1, v)));
                }
            }
            *(vec *)&sH[0][r][HO + tx * V] = hx;
            *(vec *)&sH[1][r][HO + tx * V] = hy;
            *(vec *)&sH[2][r][HO + tx * V] = hz;
            if (tx == 0) {
                // -1 column: Hz(i0-1, j) = Hz + Ch((Ex(j+1) - Ex(j)) - (Ey(i0) - Ey(i0-1)));
                //            Hy(i0-1, j) = Hy + Ch((Ez(i0) - Ez(i0-1)) - (Ex(k+1) - Ex(k)))
                T cz = xd, cy = xe;
                if (xl) {
                    const T exu = sExm[r + 1];  // Ex(i0-1, j+1); 0 beyond the domain (wall)
                    if (k >= 1)
                        cz = curl_update(xd, xchz, exu, xa0, el<T, V>(e1, 0), xb);
                    if (j >= 1)
                        cy = curl_update(xe, xchy, el<T, V>(e2, 0), xc, xa1, xa0);
                }
                sH[2][r][HO - 1] = cz;
                sH[1][r][HO - 1] = cy;
                sH[0][r][HO - 1] = 0;
            }
        }
        {
            // unconditional stores (see st_plane): a cell at i >= nx carries its loaded,
            // never-updated value (a wall or padding constant equal in both buffers)
            const unsigned so = hrow && erow && act && own ? off : kDrop;
            st_plane<T, V, NT>(dst.f[3] + pk, plane_bytes, so, hx);
            st_plane<T, V, NT>(dst.f[4] + pk, plane_bytes, so, hy);
            st_plane<T, V, NT>(dst.f[5] + pk, plane_bytes, so, hz);
        }
        __syncthreads();
        // ---------------- E^{n+1} at plane k ----------------
        vec ex = e0, ey = e1, ez = e2;
        if (erow && act && own) {
            const vec hzj = *(const vec *)&sH[2][r - 1][HO + tx * V];  // Hz(i, j-1)
            const vec hxj = *(const vec *)&sH[0][r - 1][HO + tx * V];  // Hx(i, j-1)
            const T hzl = sH[2][r][HO + tx * V - 1];                   // Hz(ib-1, j)
            const T hyl = sH[1][r][HO + tx * V - 1];                   // Hy(ib-1, j)
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int i = ib + v;
                if (i >= nx)
                    continue;
                const T hz_im = v > 0 ? el<T, V>(hz, v - 1) : hzl;
                const T hy_im = v > 0 ? el<T, V>(hy, v - 1) : hyl;
                if (j >= 1 && k >= 1)
                    set_el<T, V>(ex, v, curl_update(el<T, V>(e0, v), el<T, V>(ce0, v), el<T, V>(hz, v),
                                                    el<T, V>(hzj, v), el<T, V>(hy, v), el<T, V>(hpy, v)));
                if (i >= 1 && k >= 1)
                    set_el<T, V>(ey, v, curl_update(el<T, V>(e1, v), el<T, V>(ce1, v), el<T, V>(hx, v),
                                                    el<T, V>(hpx, v), el<T, V>(hz, v), hz_im));
                if (i >= 1 && j >= 1)
                    set_el<T, V>(ez, v, curl_update(el<T, V>(e2, v), el<T, V>(ce2, v), el<T, V>(hy, v), hy_im,
                                                    el<T, V>(hx, v), el<T, V>(hxj, v)));
            }
        }
        // driven cavity: the point source joins its E node right after the update, then the
        // probes of this plane read E; the plane tests are uniform, only the owning lane of a node
        // acts
        {
            const int lin = ib + px * j;
            const bool mine = erow && act && own;
            if (xt.sf >= 0 && k == xt.sk && mine) {
                const int d = xt.sxy - lin;
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    if (d != v)
                        continue;
                    if (xt.sf == 0)
                        set_el<T, V>(ex, v, el<T, V>(ex, v) + (T)xt.w);
                    else if (xt.sf == 1)
                        set_el<T, V>(ey, v, el<T, V>(ey, v) + (T)xt.w);
                    else
                        set_el<T, V>(ez, v, el<T, V>(ez, v) + (T)xt.w);
                }
            }
            if (xt.rec_row) {
                for (int q = 0; q < xt.pl.np; ++q) {
                    if (xt.pl.pk[q] != k)
                        continue;
                    const int d = xt.pl.pxy[q] - lin;
                    const int f = xt.pl.pf[q];
#pragma unroll
                    for (int v = 0; v < V; ++v)
                        if (mine && d == v)
                            xt.rec_row[q] = (double)(f == 0 ? el<T, V>(ex, v) : f == 1 ? el<T, V>(ey, v) : el<T, V>(ez, v));
                }
            }
        }
        {
            const unsigned so = erow && act && own ? off : kDrop;
            st_plane<T, V, NT>(dst.f[0] + pk, plane_bytes, so, ex);
            st_plane<T, V, NT>(dst.f[1] + pk, plane_bytes, so, ey);
            st_plane<T, V, NT>(dst.f[2] + pk, plane_bytes, so, ez);
        }
        // ---------------- rotate the pipeline ----------------
        hpx = hx;
        hpy = hy;
        e0 = n0;
        e1 = n1;
        e2 = n2;
        n0 = p0;
        n1 = p1;
        n2 = p2;
        ho0 = q0;
        ho1 = q1;
        ho2 = q2;
        if (CE_ARR) {
            ce0 = pce0;
            ce1 = pce1;
            ce2 = pce2;
        }
        if (CH_ARR) {
            ch0 = pch0;
            ch1 = pch1;
            ch2 = pch2;
            xchz = pxchz;
            xchy = pxchy;
        }
        xa0 = xa1;
        xa1 = pxa;
        xb = pxb;
        xc = pxc;
        xd = pxd;
        xe = pxe;
    }
}

template <typename T, int V, int R, bool NT>
hipError_t launch_cfg(const Geom &g, const Fields<T> &src, const Fields<T> &dst, const Coefs<T> &c, int zchunk,
                      hipStream_t s, const SlabExtras &xt)
{
    constexpr int TX = 64 * V;
    const int kchunk = (g.nz + zchunk - 1) / zchunk;
    const int nzc = (g.nz + kchunk - 1) / kchunk;
    const int ntx = (g.nx + TX - 1) / TX, nty = (g.ny + R - 3) / (R - 2);
    const int ntiles = ntx * nty * nzc;
    const int nblocks = (ntiles + kXcds - 1) / kXcds * kXcds;
    dim3 block(64, R), grid(nblocks);
    const bool cea = c.ce[0] != nullptr, cha = c.ch[0] != nullptr;
    if (cea && cha)
        hipLaunchKernelGGL((k_slab<T, V, R, true, true, NT>), grid, block, 0, s, g, src, dst, c, kchunk, ntx, nty,
                           ntiles, xcd_remap(), xt);
    else if (cea)
        hipLaunchKernelGGL((k_slab<T, V, R, true, false, NT>), grid, block, 0, s, g, src, dst, c, kchunk, ntx, nty,
                           ntiles, xcd_remap(), xt);
    else if (cha)
        hipLaunchKernelGGL((k_slab<T, V, R, false, true, NT>), grid, block, 0, s, g, src, dst, c, kchunk, ntx, nty,
                           ntiles, xcd_remap(), xt);
    else
        hipLaunchKernelGGL((k_slab<T, V, R, false, false, NT>), grid, block, 0, s, g, src, dst, c, kchunk, ntx, nty,
                           ntiles, xcd_remap(), xt);
    return hipGetLastError();
}

template <typename T, bool NT>
hipError_t launch_variant(const Geom &g, const Fields<T> &src, const Fields<T> &dst, const Coefs<T> &c, int zchunk,
                          int variant, hipStream_t s, const SlabExtras &xt)
{
    switch (variant) {
    case 1: return launch_cfg<T, 2, 8, NT>(g, src, dst, c, zchunk, s, xt);
    case 2: return launch_cfg<T, 1, 16, NT>(g, src, dst, c, zchunk, s, xt);
    case 3: return launch_cfg<T, 1, 8, NT>(g, src, dst, c, zchunk, s, xt);
    default: return launch_cfg<T, 2, 16, NT>(g, src, dst, c, zchunk, s, xt);
    }
}

}  // namespace

// Tile shape variants (V cells per lane, R waves per workgroup):
//   0: (2, 16)  1: (2, 8)  2: (1, 16)  3: (1, 8)
// FP64 storage (a test configuration) always uses variant 3.
int slab_rows(int variant) { return variant == 1 || variant == 3 ? 8 : 16; }

int slab_width(int variant) { return variant == 2 || variant == 3 ? 64 : 128; }

template <typename T>
hipError_t launch_slab_step(const Geom &g, const Fields<T> &src, const Fields<T> &dst, const Coefs<T> &c,
                            int zchunk, int variant, hipStream_t s, bool nt_stores, const SlabExtras *extras)
{
    zchunk = zchunk < 1 ? 1 : zchunk;
    if (sizeof(T) == 8)
        variant = 3;
    SlabExtras none{};
    none.sf = -1;
    const SlabExtras &xt = extras ? *extras : none;
    return nt_stores ? launch_variant<T, true>(g, src, dst, c, zchunk, variant, s, xt)
                     : launch_variant<T, false>(g, src, dst, c, zchunk, variant, s, xt);
}

template hipError_t launch_slab_step<float>(const Geom &, const Fields<float> &, const Fields<float> &,
                                            const Coefs<float> &, int, int, hipStream_t, bool, const SlabExtras *);
template hipError_t launch_slab_step<double>(const Geom &, const Fields<double> &, const Fields<double> &,
                                             const Coefs<double> &, int, int, hipStream_t, bool,
                                             const SlabExtras *);

}  // namespace fdtd
