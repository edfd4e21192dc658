// Temporal schedule: TS full leapfrog steps per sweep over HBM.
//
// The paper blocks only within one step (Sec. 3: tiling, sibling fusion);
// here one z-marching sweep advances the state by TS steps, so the six
// components and the coefficients cross HBM once per TS steps.
//
// Structure (per workgroup of 16 waves: an x-y tile of W own columns x
// (R - 2 TS) own rows, marching a z-chunk; the default tile is 64 x 26 for
// TS = 2, 64 x 22 for TS = 3, 64 x 20 for TS = 4):
//   - stage s = 1..TS computes step n+s on plane p_s = k - (s-1) at loop
//     index k: H^{n+s-1/2}(p_s) from E^{n+s-1} at planes p_s and p_s+1, then
//     E^{n+s}(p_s) from H^{n+s-1/2} at planes p_s and p_s-1. Stage s-1 has
//     produced E^{n+s-1}(p_s+1) earlier in the same iteration, so each stage
//     lags the previous one by exactly one plane;
//   - every stage works on the tile grown by TS cells on each side in x and
//     y (the dependency cone of TS steps); the ring of cells that see the
//     missing neighbours shrinks by one cell per stage, so the own cells of
//     the last stage are exact. Rows are overlapped: wave r owns row
//     j0 - TS + r; one extra wave holds the x-halo columns of all rows as
//     V-wide vectors, so every cell runs the same code;
//   - E of every stage and H of the current stage are exchanged through LDS
//     (one E buffer per stage, two alternating H buffers), TS + 1 barriers
//     per plane;
//   - stage-1 inputs for plane k+1 are prefetched at the top of plane k;
//     later stages take their inputs from registers of the previous stage,
//     updated in place: the registers form rings whose slots are renamed from
//     plane to plane (the loop is unrolled TS + 2 times), so no value is
//     copied when it passes from one stage to the next;
//   - a z-chunk starts TS planes early and ends TS-1 planes late so every
//     stage sees exact inputs on the planes it stores.
//   - by default one workgroup per CU takes tile numbers from a counter in
//     the solver's arena; the tile order never changes the bits.
// Walls and the region outside the domain need no per-node predicate: a
// wall-normal H sees a curl of wall-tangential E (+0, stored as +0, with -0
// wall-normal H stored as +0), H outside the domain sees only zeros and stays 0,
// and with per-node Ce arrays (0 on the walls and, as initial value and load
// result, outside the domain) a wall or outside E gets E + 0 * curl = E; per-node
// Ch arrays are 0 outside the domain in the same way. The scalar-Ce E update
// keeps its wall predicates.
// Only the last stage stores, only own cells. Arithmetic per node is
// curl_update with the operand order of every other schedule: TS sweeps of
// this kernel equal TS single steps bit for bit.
#include <algorithm>
#include <type_traits>

#include "fdtd_internal.h"
#include "storage.h"
#include "yee_update.h"

namespace fdtd {
namespace {

constexpr int kXcds = 8;

#define FDTD_GLOBAL __attribute__((address_space(1)))

__device__ __forceinline__ FDTD_GLOBAL char *uni(const void *p)
{
    const unsigned long long v = (unsigned long long)p;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return (FDTD_GLOBAL char *)(((unsigned long long)hi << 32) | lo);
}

template <typename T>
struct V2 {
    typedef T type __attribute__((ext_vector_type(2)));
};

template <typename T>
__device__ __forceinline__ typename V2<T>::type ld2(const T *plane, unsigned boff)
{
    return *(FDTD_GLOBAL const typename V2<T>::type *)(uni(plane) + boff);
}

// Two consecutive field cells of storage type S, widened to the compute type (plain
// types; compensated cells are read as loaded bits with their group's residual records).
template <typename S>
__device__ __forceinline__ typename V2<typename Store<S>::C>::type ldf(const S *plane, unsigned boff)
{
    using C = typename Store<S>::C;
    static_assert(!Store<S>::comp, "compensated cells are read by ldb and ldrec");
    if constexpr (sizeof(S) == 2) {
        const unsigned u = *(FDTD_GLOBAL const unsigned *)(uni(plane) + boff);
        const unsigned short ua = (unsigned short)(u & 0xffffu), ub = (unsigned short)(u >> 16);
        S a, b;
        __builtin_memcpy(&a, &ua, 2);
        __builtin_memcpy(&b, &ub, 2);
        typename V2<C>::type r;
        r[0] = Store<S>::widen(a);
        r[1] = Store<S>::widen(b);
        return r;
    } else {
        return *(FDTD_GLOBAL const typename V2<C>::type *)(uni(plane) + boff);
    }
}

// Buffer store of two field cells to a plane: raw buffer with the plane as its
// range, so an offset at or beyond plane_bytes is dropped by the hardware range
// check. Every lane issues the store every plane (lanes that must not write pass
// kDrop), which keeps the number of memory operations after the prefetch loads
// the same on every path; the wait for the prefetch then never covers stores.
constexpr unsigned kDrop = 0x80000000u;
constexpr int kRawBufferWord3 = 0x00020000;  // gfx9 raw buffer: 32-bit data format, no swizzle
// cache policy of the stores: non-temporal (the written state is not read again in this
// sweep), so written lines leave L2 early and the lines of the tiles' shared halos stay
constexpr int kStoreNT = 2;

template <typename S, bool NT>
__device__ __forceinline__ void st_plane(S *plane, unsigned plane_bytes, unsigned boff,
                                         const typename V2<typename Store<S>::C>::type &x)
{
    static_assert(!Store<S>::comp, "compensated cells are stored by st_group");
    constexpr int kPol = NT ? kStoreNT : 0;
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(plane, 0, (int)plane_bytes, kRawBufferWord3);
    if constexpr (sizeof(S) == 2) {
        // both cells rounded by one packed conversion
        __builtin_amdgcn_raw_buffer_store_b32(Store<S>::pack2(x[0], x[1]), r, boff, 0, kPol);
    } else if constexpr (sizeof(S) == 4) {
        __builtin_amdgcn_raw_buffer_store_b64(x, r, boff, 0, kPol);
    } else {
        __builtin_amdgcn_raw_buffer_store_b128(x, r, boff, 0, kPol);
    }
}

// Compensated storage: the two cells of the three components of a group (E or H), each
// rounded to a 16-bit pair plus residual bytes, stored as three pairs and one pair of
// residual records (rec_plane: the group's record plane, kRecBytes per cell, roff the
// lanes' record offset; dropped offsets stay dropped).
template <typename S, bool NT>
__device__ __forceinline__ void st_group(S *const f[3], unsigned plane_bytes, unsigned boff, char *rec_plane,
                                         unsigned roff, const typename V2<typename Store<S>::C>::type *x)
{
    static_assert(Store<S>::comp, "st_group stores compensated cells");
    constexpr int kPol = NT ? kStoreNT : 0;
    unsigned short q[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        unsigned hh;
        Store<S>::enc2(x[c][0], x[c][1], hh, q[c]);
        const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(f[c], 0, (int)plane_bytes, kRawBufferWord3);
        __builtin_amdgcn_raw_buffer_store_b32(hh, r, boff, 0, kPol);
    }
    // record of the first cell: the low residual bytes; of the second: the high ones
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    u2 w;
    w.x = (unsigned)(q[0] & 0xffu) | ((unsigned)(q[1] & 0xffu) << 8) | ((unsigned)(q[2] & 0xffu) << 16);
    w.y = (unsigned)(q[0] >> 8) | ((unsigned)(q[1] >> 8) << 8) | ((unsigned)(q[2] >> 8) << 16);
    const __amdgpu_buffer_rsrc_t rr =
        __builtin_amdgcn_make_buffer_rsrc(rec_plane, 0, (int)(plane_bytes / 2 * kRecBytes), kRawBufferWord3);
    __builtin_amdgcn_raw_buffer_store_b64(w, rr, roff, 0, kPol);
}

// Buffer load of two field cells of storage type S (compute type out) with the plane as the
// buffer's range: an offset at or past nrec (kDrop for a lane outside the domain, or nrec = 0
// for a plane past the chunk) reads zeros. The prefetch loads every plane this way, so it
// needs neither a branch nor registers cleared ahead of the loads.
typedef unsigned RawPair __attribute__((ext_vector_type(2)));

template <typename S>
__device__ __forceinline__ typename V2<typename Store<S>::C>::type ldb(const S *plane, unsigned nrec, unsigned boff)
{
    using C = typename Store<S>::C;
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc((void *)plane, 0, (int)nrec, kRawBufferWord3);
    if constexpr (sizeof(S) == 2) {
        const unsigned u = __builtin_amdgcn_raw_buffer_load_b32(r, boff, 0, 0);
        if constexpr (Store<S>::comp) {
            // the loaded bits as they are (decoded with the group's residual records where they
            // are first used, see dec_group), carried in an integer vector: a 16-bit pair put into a
            // float element on its own may be a denormal bit pattern, which the compiler may flush
            RawPair raw;
            raw.x = u;
            raw.y = 0u;
            return __builtin_bit_cast(typename V2<C>::type, raw);
        } else {
            const unsigned short ua = (unsigned short)(u & 0xffffu), ub = (unsigned short)(u >> 16);
            S a, b;
            __builtin_memcpy(&a, &ua, 2);
            __builtin_memcpy(&b, &ub, 2);
            typename V2<C>::type out;
            out[0] = Store<S>::widen(a);
            out[1] = Store<S>::widen(b);
            return out;
        }
    } else if constexpr (sizeof(S) == 4) {
        return __builtin_bit_cast(typename V2<C>::type, __builtin_amdgcn_raw_buffer_load_b64(r, boff, 0, 0));
    } else {
        return __builtin_bit_cast(typename V2<C>::type, __builtin_amdgcn_raw_buffer_load_b128(r, boff, 0, 0));
    }
}

// The residual records of a lane's two cells (compensated storage): one 64-bit load from the
// group's record plane (nrec 0: zeros; a dropped offset reads zeros), as loaded bits.
__device__ __forceinline__ V2<float>::type ldrec(const char *rec_plane, unsigned nrec, unsigned roff)
{
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc((void *)rec_plane, 0, (int)nrec,
                                                                       kRawBufferWord3);
    return __builtin_bit_cast(V2<float>::type, __builtin_amdgcn_raw_buffer_load_b64(r, roff, 0, 0));
}

// Decodes, in place, the three components of a compensated group loaded by ldb (16-bit pairs)
// and ldrec (records; no-op for other types): the decode waits for the loads, so it runs
// where the values are first needed, a plane after the prefetch, not where the loads issue.
template <typename S>
__device__ __forceinline__ void dec_group(typename V2<typename Store<S>::C>::type *v,
                                          const typename V2<typename Store<S>::C>::type &rec)
{
    if constexpr (Store<S>::comp) {
        const RawPair w = __builtin_bit_cast(RawPair, rec);
        float x0, x1;
        Store<S>::template dec2r<0>(__builtin_bit_cast(RawPair, v[0]).x, w.x, w.y, x0, x1);
        v[0][0] = x0;
        v[0][1] = x1;
        Store<S>::template dec2r<1>(__builtin_bit_cast(RawPair, v[1]).x, w.x, w.y, x0, x1);
        v[1][0] = x0;
        v[1][1] = x1;
        Store<S>::template dec2r<2>(__builtin_bit_cast(RawPair, v[2]).x, w.x, w.y, x0, x1);
        v[2][0] = x0;
        v[2][1] = x1;
    } else {
        (void)v;
        (void)rec;
    }
}

// Workgroup shape of the temporal sweep: 16 waves; RPW rows per wave
// (64/RPW lanes per row, 2 cells per lane); the last NHW waves hold the
// x-halo vectors of all rows.
template <int TS, int RPW>
struct TShape {
    static constexpr int V = 2;                          // cells per lane (x)
    static constexpr int LPR = 64 / RPW;                 // lanes per row
    static constexpr int W = LPR * V;                    // own columns
    static constexpr int NVH = (TS + V - 1) / V;         // halo vectors per side
    static constexpr int HX = NVH * V;                   // halo columns per side
    static constexpr int NHW = (RPW == 2 && TS >= 3) ? 2 : 1;  // halo waves
    static constexpr int NRW = 16 - NHW;                 // row waves
    static constexpr int R = NRW * RPW;                  // rows (own rows: R - 2 TS)
    static_assert(2 * NVH * R <= 64 * NHW, "halo lanes do not fit");
};

// One workgroup's tile: columns [64*tile_x ...), own rows starting at
// tile_y * (R - 2 TS), planes [zc * kchunk, ...).
template <typename S, int TS, int RPW, bool CE_ARR, bool CH_ARR, bool NT>
__device__ __forceinline__ void temporal_tile(const Geom &g, const Fields<S> &src, const Fields<S> &dst,
                                              const Coefs<typename Store<S>::C> &c, int kchunk, int tile_x,
                                              int tile_y, int zc)
{
    using T = typename Store<S>::C;  // compute type (FP32 for 16-bit storage)
    using Sh = TShape<TS, RPW>;
    constexpr int V = Sh::V, W = Sh::W, NVH = Sh::NVH, HX = Sh::HX, R = Sh::R, NRW = Sh::NRW, LPR = Sh::LPR;
    constexpr int LP = HX + W + HX + V;     // LDS row pitch (one pad vector at the end)
    constexpr int RB = R + 2;               // LDS rows (one pad row each side)
    using vec = typename V2<T>::type;
    // predicate-free E update with per-node Ce arrays (see the file header; the H update
    // never needs one)
    constexpr bool NP_E = CE_ARR;
    __shared__ __attribute__((aligned(16))) T sE[TS][3][RB][LP];  // E input of each stage, plane p_s
    __shared__ __attribute__((aligned(16))) T sH[2][3][RB][LP];   // H of the current stage (alternating)

    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const long long P = g.plane;
    const int px = g.px;
    const int i0 = tile_x * W;
    const int j0 = tile_y * (R - 2 * TS);
    const int kb = zc * kchunk;
    const int ke = min(nz, kb + kchunk);

    // zero the LDS once: pad rows and columns are read (by halo cells only) but never written
    {
        T *flatE = &sE[0][0][0][0];
        T *flatH = &sH[0][0][0][0];
        const int tid = threadIdx.y * 64 + threadIdx.x;
        for (int q = tid; q < TS * 3 * RB * LP; q += 1024) flatE[q] = 0;
        for (int q = tid; q < 2 * 3 * RB * LP; q += 1024) flatH[q] = 0;
    }

    // lane geometry: (row, first local column c0) of the lane's V cells
    const int wave = threadIdx.y, lane = threadIdx.x;
    int row, c0;
    bool lane_ok;
    const bool main_wave = wave < NRW;
    if (main_wave) {
        row = wave * RPW + lane / LPR;
        c0 = (lane % LPR) * V;
        lane_ok = true;
    } else {
        const int L = (wave - NRW) * 64 + lane;
        const int q = L % (2 * NVH);
        row = L / (2 * NVH);
        lane_ok = row < R;
        if (!lane_ok)
            row = 0;
        c0 = q < NVH ? -HX + q * V : W + (q - NVH) * V;
    }
    const int ib = i0 + c0;
    const int j = j0 - TS + row;
    const bool act = lane_ok && j >= 0 && j < ny && ib >= 0 && ib < nx;
    const bool own = main_wave && row >= TS && row < R - TS && act;
    const unsigned offs = (unsigned)(ib + px * j) * (unsigned)sizeof(S);  // field byte offset in a plane
    const unsigned offc = (unsigned)(ib + px * j) * (unsigned)sizeof(T);  // coefficient byte offset
    const int lr = row + 1;     // LDS row
    const int lc = HX + c0;     // LDS column of the first cell

    // residual record plane of a compensated group (base: Ex or Hx, whose element 0 is lo_off
    // bytes before the group's record of element 0; kRecBytes per element)
    auto rp = [&](const S *base, long long pk) { return (const char *)base + g.lo_off + kRecBytes * pk; };
    const S *Ex = src.f[0], *Ey = src.f[1], *Ez = src.f[2];
    const S *Hx = src.f[3], *Hy = src.f[4], *Hz = src.f[5];
    const vec zero = (vec)(T)0;

    // Per-stage registers live in rings indexed by a compile-time phase ph of the plane loop
    // (unrolled M times), so that a value moves from stage s to stage s+1 at the next plane by
    // a change of name, not a register copy; every update is in place.
    //   E ring roles: -2 (stage-1 E prefetched for plane k+2), -1 (E^n at p_1 + 1),
    //                 s = 0..TS-1 (E input of stage s at p_s, updated in place to its output);
    //   H ring roles: -1 (stage-1 H prefetched for plane k+1), s = 0..TS-1 (old H of stage s,
    //                 updated in place), TS (last stage's new H one plane down);
    //   coefficient rings: -1 (prefetch), s = 0..TS-1.
    // Role r of a ring sits in slot (r + off + ph) mod M; the next plane has phase ph - 1, so
    // role r becomes role r + 1 in place. Stage s's H one plane down, which its E update reads,
    // is role s+1 of the H ring before stage s+1 updates it.
    // The kernels with per-node Ch, the compensated types and plain 16-bit storage at TS = 4
    // do not unroll (their M copies spill registers): they run the ring at phase 0 and rotate
    // it by one slot after each plane, a copy of each live value, as the rename would.
    constexpr int M = TS + 2;
    constexpr bool RING = !CH_ARR && !Store<S>::comp && !(sizeof(S) == 2 && TS == 4);
    constexpr int U = RING ? M : 1;  // planes per loop iteration
    vec RE[M][3], RH[M][3], RC[M][3], RK[M][3];
    vec RRE[M], RRH[M];  // compensated storage: residual records of the E and H groups (loaded bits)
#pragma unroll
    for (int r = 0; r < M; ++r) {
        RRE[r] = zero;
        RRH[r] = zero;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            RE[r][q] = zero;
            RH[r][q] = zero;
            // per-node Ce starts at 0 where the E update has no predicates: a lane outside the
            // domain never loads it, and a zero coefficient makes its E update a no-op
            RC[r][q] = NP_E ? zero : (vec)c.ce_s;
            RK[r][q] = (vec)c.ch_s;
        }
    }
#define ES(r, ph) ((((r) + 2 + (ph)) % M + M) % M)
#define HS(r, ph) ((((r) + 1 + (ph)) % M + M) % M)

    const int k0 = max(0, kb - TS);
    const int kend = ke + TS - 2;  // last loop index
    const unsigned plane_bytes = (unsigned)(P * (long long)sizeof(S));
    const unsigned cplane_bytes = (unsigned)(P * (long long)sizeof(T));
    // first planes of stage 1, in the phase-0 slots
    if (act) {
        const long long pk = (long long)k0 * P;
        if constexpr (Store<S>::comp) {
            RE[ES(0, 0)][0] = ldb<S>(Ex + pk, plane_bytes, offs);
            RE[ES(0, 0)][1] = ldb<S>(Ey + pk, plane_bytes, offs);
            RE[ES(0, 0)][2] = ldb<S>(Ez + pk, plane_bytes, offs);
            dec_group<S>(RE[ES(0, 0)], ldrec(rp(Ex, pk), cplane_bytes, offc));
        } else {
            RE[ES(0, 0)][0] = ldf(Ex + pk, offs);
            RE[ES(0, 0)][1] = ldf(Ey + pk, offs);
            RE[ES(0, 0)][2] = ldf(Ez + pk, offs);
        }
        // E(k0+1) and H(k0) as loaded bits: the first plane decodes them like every prefetch
        const unsigned n1 = k0 + 1 < nz ? plane_bytes : 0u;
        RE[ES(-1, 0)][0] = ldb<S>(Ex + pk + P, n1, offs);
        RE[ES(-1, 0)][1] = ldb<S>(Ey + pk + P, n1, offs);
        RE[ES(-1, 0)][2] = ldb<S>(Ez + pk + P, n1, offs);
        RH[HS(0, 0)][0] = ldb<S>(Hx + pk, plane_bytes, offs);
        RH[HS(0, 0)][1] = ldb<S>(Hy + pk, plane_bytes, offs);
        RH[HS(0, 0)][2] = ldb<S>(Hz + pk, plane_bytes, offs);
        if constexpr (Store<S>::comp) {
            RRE[ES(-1, 0)] = ldrec(rp(Ex, pk + P), n1 ? cplane_bytes : 0u, offc);
            RRH[HS(0, 0)] = ldrec(rp(Hx, pk), cplane_bytes, offc);
        }
        if (CE_ARR) {
            RC[HS(0, 0)][0] = ld2(c.ce[0] + pk, offc);
            RC[HS(0, 0)][1] = ld2(c.ce[1] + pk, offc);
            RC[HS(0, 0)][2] = ld2(c.ce[2] + pk, offc);
        }
        if (CH_ARR) {
            RK[HS(0, 0)][0] = ld2(c.ch[0] + pk, offc);
            RK[HS(0, 0)][1] = ld2(c.ch[1] + pk, offc);
            RK[HS(0, 0)][2] = ld2(c.ch[2] + pk, offc);
        }
    }
    __syncthreads();  // LDS zeroing done
    // vmcnt(0): the prologue loads land in registers the loop carries; without this wait the
    // compiler's conservative merge at the loop head makes every plane wait for its own prefetch
    __builtin_amdgcn_s_waitcnt(0x0F70);
    const unsigned lfo = act ? offs : kDrop, lco = act ? offc : kDrop;  // prefetch load offsets

    for (int kk = k0; kk <= kend; kk += U) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int ph = (M - u) % M;  // a constant once unrolled: 0, M-1, ..., 1
            const int k = kk + u;
            if (k > kend)
                break;
            // residual record planes: their bases are formed per plane from the group bases (a
            // loop-invariant copy would hold more SGPRs)
            long long lo = g.lo_off;
            if constexpr (Store<S>::comp)
                __asm__ volatile("" : "+s"(lo));
            auto rp = [&](const S *base, long long pk) { return (const char *)base + lo + kRecBytes * pk; };
            auto rq = [&](S *base, long long pk) { return (char *)base + lo + kRecBytes * pk; };
            // ---------------- prefetch stage-1 inputs of plane k+1 (E of k+2) ----------------
            // (planes past the chunk or the domain, and lanes outside it, read zeros)
            {
                const bool pv = k + 1 <= kend && k + 1 < nz;
                const bool pv2 = pv && k + 2 < nz;
                const long long pk1 = pv ? (long long)(k + 1) * P : 0;
                const long long pk2 = pv2 ? pk1 + P : 0;
                const unsigned n1 = pv ? plane_bytes : 0u, n2 = pv2 ? plane_bytes : 0u, nc = pv ? cplane_bytes : 0u;
                RE[ES(-2, ph)][0] = ldb<S>(Ex + pk2, n2, lfo);
                RE[ES(-2, ph)][1] = ldb<S>(Ey + pk2, n2, lfo);
                RE[ES(-2, ph)][2] = ldb<S>(Ez + pk2, n2, lfo);
                RH[HS(-1, ph)][0] = ldb<S>(Hx + pk1, n1, lfo);
                RH[HS(-1, ph)][1] = ldb<S>(Hy + pk1, n1, lfo);
                RH[HS(-1, ph)][2] = ldb<S>(Hz + pk1, n1, lfo);
                if constexpr (Store<S>::comp) {
                    RRE[ES(-2, ph)] = ldrec(rp(Ex, pk2), n2 ? cplane_bytes : 0u, lco);
                    RRH[HS(-1, ph)] = ldrec(rp(Hx, pk1), nc, lco);
                }
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    if (CE_ARR)
                        RC[HS(-1, ph)][q] = ldb<T>(c.ce[q] + pk1, nc, lco);
                    if (CH_ARR)
                        RK[HS(-1, ph)][q] = ldb<T>(c.ch[q] + pk1, nc, lco);
                }
            }
            // compensated types: the previous plane's prefetch, decoded now (E role -1, H role 0)
            dec_group<S>(RE[ES(-1, ph)], RRE[ES(-1, ph)]);
            dec_group<S>(RH[HS(0, ph)], RRH[HS(0, ph)]);
            // ---------------- stage the E input of every stage ----------------
            if (lane_ok) {
#pragma unroll
                for (int s = 0; s < TS; ++s)
#pragma unroll
                    for (int q = 0; q < 3; ++q) *(vec *)&sE[s][q][lr][lc] = RE[ES(s, ph)][q];
            }
            __syncthreads();

#pragma unroll
            for (int s = 0; s <= TS; ++s) {
                // ---- E update of stage s-1 (its H was staged in the previous phase) ----
                if (s > 0) {
                    const int sp = s - 1;
                    const int pp = k - sp;
                    const int lop = sp == TS - 1 ? max(0, kb - 1) : max(0, kb - TS + sp);
                    const int hip = sp == TS - 1 ? ke - 1 : min(nz - 1, ke + TS - 2 - sp);
                    const bool livep = pp >= lop && pp <= hip;
                    const int hb = (sp + 1) & 1;
                    vec *E = RE[ES(sp, ph)];
                    const vec *Hn = RH[HS(sp, ph)];      // H^{n+sp+1/2}(p_sp), just updated
                    const vec *Hd = RH[HS(sp + 1, ph)];  // the same H one plane down
                    const vec *Cs = RC[HS(sp, ph)];
                    if (livep && (NP_E || act)) {
                        const vec hzj = *(const vec *)&sH[hb][2][lr - 1][lc];  // Hz(i, j-1)
                        const vec hxj = *(const vec *)&sH[hb][0][lr - 1][lc];  // Hx(i, j-1)
                        const T hzl = sH[hb][2][lr][lc - 1];                   // Hz(ib-1, j)
                        const T hyl = sH[hb][1][lr][lc - 1];                   // Hy(ib-1, j)
#pragma unroll
                        for (int v = 0; v < V; ++v) {
                            const int i = ib + v;
                            if (!NP_E && i >= nx)
                                continue;
                            const T hz_im = v > 0 ? Hn[2][v - 1] : hzl;
                            const T hy_im = v > 0 ? Hn[1][v - 1] : hyl;
                            if (NP_E || (j >= 1 && pp >= 1))
                                E[0][v] = curl_update(E[0][v], Cs[0][v], Hn[2][v], hzj[v], Hn[1][v], Hd[1][v]);
                            if (NP_E || (i >= 1 && pp >= 1))
                                E[1][v] = curl_update(E[1][v], Cs[1][v], Hn[0][v], Hd[0][v], Hn[2][v], hz_im);
                            if (NP_E || (i >= 1 && j >= 1))
                                E[2][v] = curl_update(E[2][v], Cs[2][v], Hn[1][v], hy_im, Hn[0][v], hxj[v]);
                        }
                    }
                    if (sp < TS - 1 && !livep) {
                        E[0] = zero;
                        E[1] = zero;
                        E[2] = zero;
                    }
                    if (sp == TS - 1) {
                        // unconditional stores (see st_plane); the cell at i = nx of a lane whose
                        // second cell leaves the domain carries its loaded, never-updated value (a
                        // wall or padding constant equal in both buffers), so storing both cells
                        // is exact
                        const bool wr = livep && own && pp >= kb;
                        const unsigned so = wr ? offs : kDrop;
                        const long long pk = (long long)(pp > 0 ? pp : 0) * P;
                        if constexpr (Store<S>::comp) {
                            const unsigned sor = wr ? offc : kDrop;  // record offset
                            S *const fe[3] = {dst.f[0] + pk, dst.f[1] + pk, dst.f[2] + pk};
                            S *const fh[3] = {dst.f[3] + pk, dst.f[4] + pk, dst.f[5] + pk};
                            st_group<S, NT>(fe, plane_bytes, so, rq(dst.f[0], pk), sor, E);
                            st_group<S, NT>(fh, plane_bytes, so, rq(dst.f[3], pk), sor, Hn);
                        } else {
                            st_plane<S, NT>(dst.f[0] + pk, plane_bytes, so, E[0]);
                            st_plane<S, NT>(dst.f[1] + pk, plane_bytes, so, E[1]);
                            st_plane<S, NT>(dst.f[2] + pk, plane_bytes, so, E[2]);
                            st_plane<S, NT>(dst.f[3] + pk, plane_bytes, so, Hn[0]);
                            st_plane<S, NT>(dst.f[4] + pk, plane_bytes, so, Hn[1]);
                            st_plane<S, NT>(dst.f[5] + pk, plane_bytes, so, Hn[2]);
                        }
                    }
                }
                if (s == TS)
                    break;
                // ---- H update of stage s, in place ----
                const int p = k - s;  // plane of stage s+1
                const int lo = max(0, kb - TS + s), hi = min(nz - 1, ke + TS - 2 - s);
                const bool live = p >= lo && p <= hi;
                const vec *en = RE[ES(s - 1, ph)];  // E input at plane p+1 (own column): role -1 or stage s-1's output
                const vec *Es = RE[ES(s, ph)];
                const vec *Ks = RK[HS(s, ph)];
                vec *H = RH[HS(s, ph)];
                const int hb = (s + 1) & 1;
                if (live) {
                    const vec ezj = *(const vec *)&sE[s][2][lr + 1][lc];  // Ez(i, j+1)
                    const vec exj = *(const vec *)&sE[s][0][lr + 1][lc];  // Ex(i, j+1)
                    const T ezr = sE[s][2][lr][lc + V];                    // Ez(ib+V, j)
                    const T eyr = sE[s][1][lr][lc + V];                    // Ey(ib+V, j)
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        const T ez_ip = v + 1 < V ? Es[2][v + 1] : ezr;
                        const T ey_ip = v + 1 < V ? Es[1][v + 1] : eyr;
                        H[0][v] = curl_update(H[0][v], Ks[0][v], en[1][v], Es[1][v], ezj[v], Es[2][v]);
                        H[1][v] = curl_update(H[1][v], Ks[1][v], ez_ip, Es[2][v], en[0][v], Es[0][v]);
                        H[2][v] = curl_update(H[2][v], Ks[2][v], exj[v], Es[0][v], ey_ip, Es[1][v]);
                    }
                }
                if (lane_ok) {
                    *(vec *)&sH[hb][0][lr][lc] = H[0];
                    *(vec *)&sH[hb][1][lr][lc] = H[1];
                    *(vec *)&sH[hb][2][lr][lc] = H[2];
                }
                __syncthreads();
            }
            if (!RING) {
                // role r moves to role r + 1: every ring shifts one slot up (the values that
                // wrap round are dead: the next prefetch overwrites them)
#pragma unroll
                for (int r = M - 1; r > 0; --r)
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        RE[r][q] = RE[r - 1][q];
                        RH[r][q] = RH[r - 1][q];
                        RC[r][q] = RC[r - 1][q];
                        RK[r][q] = RK[r - 1][q];
                    }
                if constexpr (Store<S>::comp)
#pragma unroll
                    for (int r = M - 1; r > 0; --r) {
                        RRE[r] = RRE[r - 1];
                        RRH[r] = RRH[r - 1];
                    }
            }
        }
    }
#undef ES
#undef HS
}

// Tile number of virtual block v (with one workgroup per tile, v is the
// hardware block number, and block b runs on XCD b % 8).
// remap 1: XCD x owns tiles [x * nper, (x + 1) * nper).
// remap 2: one workgroup per CU is resident, so blocks 8 cpx w .. 8 cpx (w + 1) - 1
// run together; they take the contiguous tile range starting at 8 cpx w, XCD x
// the x-th part of it, so the halo rows two neighbouring parts share are read
// at about the same time (the last, partial range is split the same way).
__device__ __forceinline__ int tile_of_block(int v, int ntiles, int remap, int cpx)
{
    if (remap == 0)
        return v;
    const int x = v % kXcds, k = v / kXcds;
    if (remap == 1)
        return x * ((ntiles + kXcds - 1) / kXcds) + k;
    const int w = k / cpx, base = w * kXcds * cpx;
    const int rem = min(kXcds * cpx, ntiles - base);
    return base + x * ((rem + kXcds - 1) / kXcds) + (k - w * cpx);
}

// Tile queue: one workgroup per CU takes virtual blocks until none is left.
// Virtual block v (v < nvb, a multiple of 8) sits in list v % 8, in the
// remap-2 order above; the workgroups on XCD x (hardware register XCC_ID) take
// list x in order, so the tiles that share halo lines run together in one L2,
// then help the other lists, so every block is taken exactly once wherever the
// workgroups run. A CU that ends a tile early starts the next at once, instead
// of waiting for the dispatcher, which hands out blocks in order round the
// XCDs and so holds every XCD to the slowest. No workgroup ever waits for
// another. q[0..7]: next index of each list; q[8]: workgroups done; q[9]: lists
// seen empty. The one that finishes last has seen every take and zeroes the
// counters for the next launch (launches sharing them are ordered by their stream).
constexpr int kQueueWords = kXcds + 2;

struct TileQueue {
    unsigned *q;
    int per;   // blocks per list (nvb / 8)
    int list;  // list taken now

    __device__ explicit TileQueue(unsigned *q_, int nvb) : q(q_), per(nvb / kXcds)
    {
        unsigned xcc;
        asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(xcc));
        list = (int)(xcc & (kXcds - 1));
    }
    // Next virtual block, or -1 when every list is empty (lead lane only). A take
    // that finds its list empty sets the list's bit in q[9], which then names the
    // lists every workgroup has seen empty: the workgroup moves to one without a
    // bit, and leaves when all eight are set. Each list sends a workgroup on at
    // most once, so the loop ends.
    __device__ int take()
    {
        for (;;) {
            const int j = (int)atomicAdd(&q[list], 1u);
            if (j < per)
                return j * kXcds + list;
            const unsigned empty = atomicOr(&q[kXcds + 1], 1u << list) | (1u << list);
            if (empty == 0xffu)
                return -1;
            list = __ffs(~empty) - 1;
        }
    }
    __device__ void finish()
    {
        if (atomicAdd(&q[kXcds], 1u) == gridDim.x - 1)
            for (int i = 0; i < kQueueWords; ++i)
                atomicExch(&q[i], 0u);
    }
};

template <typename S, int TS, int RPW, bool CE_ARR, bool CH_ARR, bool NT>
__global__ void __launch_bounds__(1024)
    k_temporal(Geom g, Fields<S> src, Fields<S> dst, Coefs<typename Store<S>::C> c, int kchunk, int ntx, int nty,
               int ntiles, int remap, int cpx)
{
    const int t = tile_of_block(blockIdx.x, ntiles, remap, cpx);
    if (t >= ntiles)
        return;  // the whole workgroup leaves before any barrier
    temporal_tile<S, TS, RPW, CE_ARR, CH_ARR, NT>(g, src, dst, c, kchunk, t % ntx, (t / ntx) % nty, t / (ntx * nty));
}

// Queue schedule (TileQueue above).
template <typename S, int TS, int RPW, bool CE_ARR, bool CH_ARR, bool NT>
__global__ void __launch_bounds__(1024)
    k_temporal_q(Geom g, Fields<S> src, Fields<S> dst, Coefs<typename Store<S>::C> c, int kchunk, int ntx, int nty,
                 int ntiles, int nvb, int cpx, unsigned *queue)
{
    __shared__ int s_v;
    const bool lead = threadIdx.x == 0 && threadIdx.y == 0;
    TileQueue tq(queue, nvb);
    for (;;) {
        if (lead)
            s_v = tq.take();
        __syncthreads();
        const int v = s_v;
        __syncthreads();  // every lane has read s_v before the next take rewrites it
        if (v < 0)
            break;  // the same for the whole workgroup
        const int t = tile_of_block(v, ntiles, 2, cpx);
        if (t < ntiles)
            temporal_tile<S, TS, RPW, CE_ARR, CH_ARR, NT>(g, src, dst, c, kchunk, t % ntx, (t / ntx) % nty,
                                                          t / (ntx * nty));
        __syncthreads();  // the next tile rewrites the LDS this one read last
    }
    if (lead)
        tq.finish();
}

// One launch over the tiles of several cavities (continuous batching): the
// tile number picks the request (entries sorted by tile_begin), then the
// request's own geometry, buffers and coefficients run the same tile code as
// a single solve, so each request's bits do not depend on the batch.
template <int TS, bool CE_ARR, bool CH_ARR>
__device__ __forceinline__ void batch_tile(const BatchEntry *__restrict__ table, int nreq, int t)
{
    int lo = 0, hi = nreq - 1;  // last entry with tile_begin <= t
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (table[mid].tile_begin <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    const BatchEntry e = table[lo];
    const int u = t - e.tile_begin;
    temporal_tile<float, TS, 2, CE_ARR, CH_ARR, true>(e.g, e.src, e.dst, e.c, e.kchunk, u % e.ntx, (u / e.ntx) % e.nty,
                                                u / (e.ntx * e.nty));
}

template <int TS, bool CE_ARR, bool CH_ARR>
__global__ void __launch_bounds__(1024)
    k_temporal_batch(const BatchEntry *__restrict__ table, int nreq, int ntiles, int remap, int cpx)
{
    const int t = tile_of_block(blockIdx.x, ntiles, remap, cpx);
    if (t >= ntiles)
        return;
    batch_tile<TS, CE_ARR, CH_ARR>(table, nreq, t);
}

// The batched launch with the tile queue of k_temporal_q (the pool's own counters).
template <int TS, bool CE_ARR>
__global__ void __launch_bounds__(1024)
    k_temporal_batch_q(const BatchEntry *__restrict__ table, int nreq, int ntiles, int nvb, int cpx, unsigned *queue)
{
    __shared__ int s_v;
    const bool lead = threadIdx.x == 0 && threadIdx.y == 0;
    TileQueue tq(queue, nvb);
    for (;;) {
        if (lead)
            s_v = tq.take();
        __syncthreads();
        const int v = s_v;
        __syncthreads();
        if (v < 0)
            break;
        const int t = tile_of_block(v, ntiles, 2, cpx);
        if (t < ntiles)
            batch_tile<TS, CE_ARR, false>(table, nreq, t);
        __syncthreads();
    }
    if (lead)
        tq.finish();
}

template <typename T, int TS, int RPW, bool NT>
hipError_t launch_ts(const Geom &g, const Fields<T> &src, const Fields<T> &dst,
                     const Coefs<typename Store<T>::C> &c, int zchunk, hipStream_t s, unsigned *queue)
{
    using Sh = TShape<TS, RPW>;
    const int kchunk = (g.nz + zchunk - 1) / zchunk;
    const int nzc = (g.nz + kchunk - 1) / kchunk;
    const int own = Sh::R - 2 * TS;
    const int ntx = (g.nx + Sh::W - 1) / Sh::W, nty = (g.ny + own - 1) / own;
    const int ntiles = ntx * nty * nzc;
    const int cpx = cus_per_xcd();
    dim3 block(64, 16);
    const bool cea = c.ce[0] != nullptr, cha = c.ch[0] != nullptr;
    if (queue && temporal_sched() == 1) {
        const int nvb = (ntiles + kXcds - 1) / kXcds * kXcds;
        dim3 grid(std::min(ntiles, kXcds * cpx));  // one workgroup per CU
        if (cea && cha)
            hipLaunchKernelGGL((k_temporal_q<T, TS, RPW, true, true, NT>), grid, block, 0, s, g, src, dst, c, kchunk,
                               ntx, nty, ntiles, nvb, cpx, queue);
        else if (cha)
            hipLaunchKernelGGL((k_temporal_q<T, TS, RPW, false, true, NT>), grid, block, 0, s, g, src, dst, c, kchunk,
                               ntx, nty, ntiles, nvb, cpx, queue);
        else if (cea)
            hipLaunchKernelGGL((k_temporal_q<T, TS, RPW, true, false, NT>), grid, block, 0, s, g, src, dst, c, kchunk,
                               ntx, nty, ntiles, nvb, cpx, queue);
        else
            hipLaunchKernelGGL((k_temporal_q<T, TS, RPW, false, false, NT>), grid, block, 0, s, g, src, dst, c, kchunk,
                               ntx, nty, ntiles, nvb, cpx, queue);
        return hipGetLastError();
    }
    const int nblocks = (ntiles + kXcds - 1) / kXcds * kXcds;
    dim3 grid(nblocks);
    const int rm = xcd_remap();
    if (cea && cha)
        hipLaunchKernelGGL((k_temporal<T, TS, RPW, true, true, NT>), grid, block, 0, s, g, src, dst, c, kchunk, ntx, nty,
                           ntiles, rm, cpx);
    else if (cea)
        hipLaunchKernelGGL((k_temporal<T, TS, RPW, true, false, NT>), grid, block, 0, s, g, src, dst, c, kchunk, ntx,
                           nty, ntiles, rm, cpx);
    else if (cha)
        hipLaunchKernelGGL((k_temporal<T, TS, RPW, false, true, NT>), grid, block, 0, s, g, src, dst, c, kchunk, ntx,
                           nty, ntiles, rm, cpx);
    else
        hipLaunchKernelGGL((k_temporal<T, TS, RPW, false, false, NT>), grid, block, 0, s, g, src, dst, c, kchunk, ntx,
                           nty, ntiles, rm, cpx);
    return hipGetLastError();
}

template <typename T, bool NT>
hipError_t launch_shape(const Geom &g, const Fields<T> &src, const Fields<T> &dst,
                        const Coefs<typename Store<T>::C> &c, int zchunk, int ts, int variant, hipStream_t s,
                        unsigned *queue)
{
    if (variant == 1) {
        switch (ts) {
        case 1: return launch_ts<T, 1, 1, NT>(g, src, dst, c, zchunk, s, queue);
        case 2: return launch_ts<T, 2, 1, NT>(g, src, dst, c, zchunk, s, queue);
        case 3: return launch_ts<T, 3, 1, NT>(g, src, dst, c, zchunk, s, queue);
        default: return hipErrorInvalidValue;
        }
    }
    switch (ts) {
    case 1: return launch_ts<T, 1, 2, NT>(g, src, dst, c, zchunk, s, queue);
    case 2: return launch_ts<T, 2, 2, NT>(g, src, dst, c, zchunk, s, queue);
    case 3: return launch_ts<T, 3, 2, NT>(g, src, dst, c, zchunk, s, queue);
    case 4: return launch_ts<T, 4, 2, NT>(g, src, dst, c, zchunk, s, queue);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

// variant 0: two rows per wave (64 x ~26 tiles, TS = 1..4); variant 1: one row per wave
// (128 x ~11 tiles, TS = 1..3)
int temporal_own_rows(int ts, int variant)
{
    return variant == 1 ? 15 - 2 * ts : (ts >= 3 ? 28 : 30) - 2 * ts;
}

int temporal_width(int variant) { return variant == 1 ? 128 : 64; }

void temporal_tiling(const Geom &g, int ts, int zchunk, int *kchunk, int *ntx, int *nty, int *ntiles)
{
    const int own = temporal_own_rows(ts, 0), w = temporal_width(0);
    zchunk = zchunk < 1 ? 1 : zchunk;
    *kchunk = (g.nz + zchunk - 1) / zchunk;
    const int nzc = (g.nz + *kchunk - 1) / *kchunk;
    *ntx = (g.nx + w - 1) / w;
    *nty = (g.ny + own - 1) / own;
    *ntiles = *ntx * *nty * nzc;
}


hipError_t launch_temporal_batch(const BatchEntry *table, int nreq, int ntiles, int ts, bool ce_arr, bool ch_arr,
                                 hipStream_t s, unsigned *queue)
{
    if (nreq <= 0 || ntiles <= 0)
        return hipSuccess;
    if (queue && !ch_arr && temporal_sched() == 1) {
        const int cpx = cus_per_xcd(), nvb = (ntiles + kXcds - 1) / kXcds * kXcds;
        dim3 block(64, 16), grid(std::min(ntiles, kXcds * cpx));
#define FDTD_BATCH_Q(TSV)                                                                                          \
    do {                                                                                                           \
        if (ce_arr)                                                                                                \
            hipLaunchKernelGGL((k_temporal_batch_q<TSV, true>), grid, block, 0, s, table, nreq, ntiles, nvb, cpx, queue);  \
        else                                                                                                       \
            hipLaunchKernelGGL((k_temporal_batch_q<TSV, false>), grid, block, 0, s, table, nreq, ntiles, nvb, cpx, queue); \
    } while (0)
        switch (ts) {
        case 1: FDTD_BATCH_Q(1); break;
        case 2: FDTD_BATCH_Q(2); break;
        case 3: FDTD_BATCH_Q(3); break;
        case 4: FDTD_BATCH_Q(4); break;
        default: return hipErrorInvalidValue;
        }
#undef FDTD_BATCH_Q
        return hipGetLastError();
    }
    const int nblocks = (ntiles + kXcds - 1) / kXcds * kXcds;
    dim3 block(64, 16), grid(nblocks);
    const int rm = xcd_remap(), cpx = cus_per_xcd();
#define FDTD_BATCH_LAUNCH(TSV, CEV, CHV) \
    hipLaunchKernelGGL((k_temporal_batch<TSV, CEV, CHV>), grid, block, 0, s, table, nreq, ntiles, rm, cpx)
#define FDTD_BATCH_TS(TSV)                                    \
    do {                                                      \
        if (ce_arr && ch_arr) FDTD_BATCH_LAUNCH(TSV, true, true);   \
        else if (ce_arr) FDTD_BATCH_LAUNCH(TSV, true, false);       \
        else if (ch_arr) FDTD_BATCH_LAUNCH(TSV, false, true);       \
        else FDTD_BATCH_LAUNCH(TSV, false, false);                  \
    } while (0)
    switch (ts) {
    case 1: FDTD_BATCH_TS(1); break;
    case 2: FDTD_BATCH_TS(2); break;
    case 3: FDTD_BATCH_TS(3); break;
    case 4: FDTD_BATCH_TS(4); break;
    default: return hipErrorInvalidValue;
    }
#undef FDTD_BATCH_TS
#undef FDTD_BATCH_LAUNCH
    return hipGetLastError();
}


template <typename T>
hipError_t launch_temporal_step(const Geom &g, const Fields<T> &src, const Fields<T> &dst,
                                const Coefs<typename Store<T>::C> &c, int zchunk, int ts, int variant,
                                hipStream_t s, bool nt_stores, unsigned *queue)
{
    zchunk = zchunk < 1 ? 1 : zchunk;
    // the default-policy stores are built for FP32 fields only (the small, cache-resident
    // states that profit from them are FP32 in practice)
    if constexpr (std::is_same<T, float>::value)
        if (!nt_stores)
            return launch_shape<T, false>(g, src, dst, c, zchunk, ts, variant, s, queue);
    (void)nt_stores;
    return launch_shape<T, true>(g, src, dst, c, zchunk, ts, variant, s, queue);
}


template hipError_t launch_temporal_step<float>(const Geom &, const Fields<float> &, const Fields<float> &,
                                                const Coefs<float> &, int, int, int, hipStream_t, bool, unsigned *);



template hipError_t launch_temporal_step<f16>(const Geom &, const Fields<f16> &, const Fields<f16> &,
                                              const Coefs<float> &, int, int, int, hipStream_t, bool, unsigned *);




template hipError_t launch_temporal_step<bf16>(const Geom &, const Fields<bf16> &, const Fields<bf16> &,
                                               const Coefs<float> &, int, int, int, hipStream_t, bool, unsigned *);



template hipError_t launch_temporal_step<f16c>(const Geom &, const Fields<f16c> &, const Fields<f16c> &,
                                               const Coefs<float> &, int, int, int, hipStream_t, bool, unsigned *);

template hipError_t launch_temporal_step<bf16c>(const Geom &, const Fields<bf16c> &, const Fields<bf16c> &,
                                                const Coefs<float> &, int, int, int, hipStream_t, bool, unsigned *);


}  // namespace fdtd

namespace fdtd {

// FP64 storage has no temporal kernel (its LDS tiles would not fit); create rejects it.
template <>
hipError_t launch_temporal_step<double>(const Geom &, const Fields<double> &, const Fields<double> &,
                                        const Coefs<double> &, int, int, int, hipStream_t, bool, unsigned *)
{
    return hipErrorNotSupported;
}

}  // namespace fdtd
