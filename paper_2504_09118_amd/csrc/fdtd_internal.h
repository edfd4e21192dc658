// Internal types of libfdtd: device layout, kernel argument packs, launchers.
//
// Device layout. Every component (Ex, Ey, Ez, Hx, Hy, Hz, and the per-node
// coefficients) lives in its own padded box of px * py * pz elements,
// x-fastest: element (i, j, k) at base[i + px * (j + py * k)], with
// px >= nx + 1 a multiple of 64 elements (each 64-lane row segment is one
// aligned 256-byte access), py = ny + 1, pz = nz + 1. Entries outside a
// component's staggered extent are padding (zero, never written). Each box
// starts on a 256-byte boundary after a 256-byte guard.
//
// Update domain. Every update of the method lies in the nx*ny*nz cell set
// (i, j, k) in [0,nx) x [0,ny) x [0,nz); per cell:
//   Hx if i >= 1, Hy if j >= 1, Hz if k >= 1   (wall-normal H never changes)
//   Ex if j, k >= 1, Ey if i, k >= 1, Ez if i, j >= 1   (PEC walls never change)
// and every value the updates read at index nx, ny or nz (x, y, z) is a
// wall-tangential E node, i.e. exactly 0. Kernels therefore index only the
// cell domain and substitute 0 beyond it.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "storage.h"

namespace fdtd {

struct Geom {
    int nx, ny, nz;
    int px, py, pz;
    long long plane;  // px * py
    long long box;    // elements reserved per component box (incl. guards, 64-aligned)
    // compensated 16-bit storage (0 otherwise): the residual records of the E components
    // sit in Ex's box after its 16-bit values, those of H in Hx's box; lo_off is the byte
    // distance from Ex's (Hx's) element 0 to the record of element 0, and lo_step + 1 the
    // distance between the boxes of one state (Ey = Ex + lo_step + 1 bytes, and so on)
    long long lo_off;
    long long lo_step;
    // byte distance from component q's element 0 to its residual byte of element 0
    __host__ __device__ long long lo_rec(int q) const { return lo_off - (long long)(q % 3) * lo_step; }
    __host__ __device__ long long at(int i, int j, int k) const
    {
        return (long long)i + (long long)px * ((long long)j + (long long)py * k);
    }
};

constexpr int kGuardElems = 64;

template <typename T>
struct Fields {
    T *f[6];  // Ex, Ey, Ez, Hx, Hy, Hz: element (0,0,0) of each box
};

template <typename T>
struct Coefs {
    const T *ce[3];  // per-node Ce boxes, or nullptr when scalar
    const T *ch[3];  // per-node Ch boxes, or nullptr when scalar
    T ce_s;          // scalar Ce (interior E nodes) when ce[] is null
    T ch_s;          // scalar Ch (non-wall H nodes) when ch[] is null
};

// Kernel schedules (values match fdtd_kernel in include/fdtd.h).
enum Schedule { kAuto = 0, kPlain = 1, kFused = 2, kSlab = 3, kTemporal = 4 };

// ---- launchers (each returns the first HIP error it meets) ----

// Plain two-sweep step, in place on f.
template <typename T>
hipError_t launch_plain_step(const Geom &g, const Fields<T> &f, const Coefs<T> &c, hipStream_t s);

// Fused one-sweep step: reads src, writes dst (src is not modified).
template <typename T>
hipError_t launch_fused_step(const Geom &g, const Fields<T> &src, const Fields<T> &dst,
                             const Coefs<T> &c, int zchunk, hipStream_t s);

// Up to kInlineProbes probe nodes carried in a sweep's kernel arguments (probe order kept):
// component pf, plane pk and in-plane element offset pxy of each.
constexpr int kInlineProbes = 16;
struct ProbeList {
    int np;
    int pf[kInlineProbes], pk[kInlineProbes], pxy[kInlineProbes];
};

// Driven-cavity extras a slab sweep can apply (the adjoint's forward and recompute): add w to
// the E node (component sf, plane sk, in-plane element offset sxy) right after its update
// (sf < 0: none), then record E of each probe q as a double in rec_row[q] (rec_row null or
// no probes: none).
struct SlabExtras {
    int sf, sk, sxy;
    double w;
    ProbeList pl;
    double *rec_row;
};

// Slab step (fused sweep with V-wide lanes, prefetch and XCD-aware tiles):
// reads src, writes dst. variant selects the tile shape (0 = default).
// nt_stores: store the new state with the non-temporal cache policy (right when
// the streamed state is larger than the last-level cache; see kStreamCacheBytes).
template <typename T>
hipError_t launch_slab_step(const Geom &g, const Fields<T> &src, const Fields<T> &dst,
                            const Coefs<T> &c, int zchunk, int variant, hipStream_t s, bool nt_stores = true,
                            const SlabExtras *extras = nullptr);

// Temporal step: ts (1..3) leapfrog steps in one sweep; reads src, writes dst.
// Built for FP32, FP16 and BF16 field storage (16-bit fields compute in FP32
// with FP32 coefficients).
// nt_stores as for the slab step (honoured for FP32 fields; 16-bit fields always
// store non-temporally).
// queue: the solver's two scheduling counters (zero before the launch, zero
// again after it), used when the tiles are handed out from a queue; may be null.
template <typename T>
hipError_t launch_temporal_step(const Geom &g, const Fields<T> &src, const Fields<T> &dst,
                                const Coefs<typename Store<T>::C> &c, int zchunk, int ts, int variant,
                                hipStream_t s, bool nt_stores = true, unsigned *queue = nullptr);

// MI355X's Infinity Cache (256 MB, the last level before HBM). A sweep whose streamed
// bytes (both state buffers and the coefficient arrays) fit in it keeps the default
// store policy, so the next sweep reads the state from the cache; larger states store
// non-temporally, which leaves L2 to the halo lines neighbouring tiles share.
constexpr size_t kStreamCacheBytes = (size_t)256 << 20;
// 32-bit scheduling counters a queue-scheduled temporal launch uses (zero before the
// launch, zero again after it): one next-tile index per XCD list, the count of finished
// workgroups and the mask of lists seen empty.
constexpr int kSchedWords = 10;
int temporal_own_rows(int ts, int variant);
int temporal_width(int variant);

// One request of a batched temporal launch (FP32 fields, variant-0 tiles).
struct BatchEntry {
    Geom g;
    Fields<float> src, dst;
    Coefs<float> c;
    int kchunk, ntx, nty, ntiles;
    int tile_begin;  // first tile of this request in the launch
};

// Tiling of one request for the batched temporal launch.
void temporal_tiling(const Geom &g, int ts, int zchunk, int *kchunk, int *ntx, int *nty, int *ntiles);

// One launch advancing every request of a device table by ts steps; entries
// sorted by tile_begin, ntiles = total tiles. All entries share ts and the
// presence of Ce / Ch arrays. queue: two scheduling counters as for
// launch_temporal_step (zero before and after), or null.
hipError_t launch_temporal_batch(const BatchEntry *table, int nreq, int ntiles, int ts, bool ce_arr, bool ch_arr,
                                 hipStream_t s, unsigned *queue = nullptr);

// Device memory plan of one cavity inside an arena (offsets from a 256-byte
// aligned base): two state buffers of six boxes, optional per-node Ce / Ch
// boxes, and (with aux) an FP64 staging array and the diagnostic partials.
struct Plan {
    Geom g;
    size_t fesz, cesz;  // bytes per field element, per coefficient element
    size_t fbox_bytes, cbox_bytes;
    size_t off_fields[2][6];
    size_t off_ce[3], off_ch[3];
    size_t off_staging, staging_bytes;  // SIZE_MAX / 0 without aux
    size_t off_diag;
    size_t off_sched;  // 256 bytes of scheduling counters (zero between launches)
    size_t total;
};

// fesz: 8, 4 or 2 bytes; coefficients are FP64 for FP64 fields, else FP32. comp: each
// field box also has room for a box of residual records (compensated 16-bit storage;
// the E records use Ex's, the H records Hx's, see Geom::lo_off).
Plan make_plan(int nx, int ny, int nz, int fesz, bool ce_arr, bool ch_arr, bool aux, bool comp = false);

// Seeded random state (E ~ U[-1,1] from a counter-based SplitMix64, PEC walls,
// H = 0) written into both state buffers a and b (b may hold nullptrs).
template <typename T>
hipError_t launch_init_random(const Geom &g, unsigned long long seed, T *const a[6], T *const b[6], hipStream_t s,
                              const double *scale = nullptr);

// Driven-cavity adjoint (FP32 / FP64 storage). Point source: add w to node
// so of component sf (sf < 0: none); probes: record E at (pf, po) into
// rec_row and add their squares to *J (rec_row null: no probes).
template <typename T>
hipError_t launch_source_probe(const Fields<T> &f, int sf, long long so, double w, int np, const int *pf,
                               const long long *po, double *rec_row, double *J, hipStream_t s);
// J = sum over rows 1..nrows of rec (np values a row) of the row's sum of squares, in probe
// and row order (the bits of adding one row per step); 1 <= np <= 4096.
hipError_t launch_probe_objective(const double *rec, long long nrows, int np, double *J, hipStream_t s);
// lam += 2 rec_row at the probe nodes.
template <typename T>
hipError_t launch_adj_probe(const Fields<T> &lam, int np, const int *pf, const long long *po, const double *rec_row,
                            hipStream_t s);
// One reverse step: a = (lam Ex Ey Ez, mu Hx Hy Hz); hist = H^{n+1/2}; gce += lam (L hist).
// gpart (null: gce directly): FP32 group sums (boxes like gce, zero at a group's start)
// that collect the term; close_group adds them to gce and clears them.
constexpr int kAdjGroup = 16;
template <typename T>
hipError_t launch_adj_step(const Geom &g, const Fields<T> &a, const Coefs<T> &c, const T *const hist[3],
                           double *const gce[3], float *const gpart[3], bool close_group, hipStream_t s);
// The fused reverse step (one z-marching sweep): reads a = (lam, mu) from src, writes
// (lam', mu') to dst; gCe as launch_adj_step; then lam' += 2 rec_row[q] at the probes of pl
// (rec_row null: none). The bits of launch_adj_step followed by launch_adj_probe. zchunk:
// z-chunks as the slab sweep.
template <typename T>
hipError_t launch_adj_sweep(const Geom &g, const Fields<T> &src, const Fields<T> &dst, const Coefs<T> &c,
                            const T *const hist[3], double *const gce[3], float *const gpart[3], bool close_group,
                            const ProbeList &pl, const double *rec_row, int zchunk, hipStream_t s);
// dJ/d eps per cell (dense x-fastest nx*ny*nz doubles) from dJ/dCe per edge.
template <typename T>
hipError_t launch_grad_eps(const Geom &g, const Coefs<T> &c, double *const gce[3], double dx_over_dt, double *out,
                           hipStream_t s);

// Tile rows owned per workgroup (rows - 2) and tile width of a slab variant.
int slab_rows(int variant);
int slab_width(int variant);

// FP64 coefficient precompute. eps / mu: device per-cell arrays (nx*ny*nz,
// x-fastest) or nullptr for 1. Writes the three boxes of each kind that are
// non-null: dt / (dx * mean) times fac[f] (fac: six per-component factors of
// rectangular cells, Ex Ey Ez Hx Hy Hz; nullptr for cubic cells).
template <typename T>
hipError_t launch_coef(const Geom &g, double dx, double dt, const double *eps, const double *mu,
                       T *ce[3], T *ch[3], hipStream_t s, const double *fac = nullptr);

// Dense staggered buffer (type S) -> padded box (type T) for field f, each
// value multiplied by scale in FP64 and rounded once; writes both destinations
// (dst2 may be null). E fields get 0 on wall-tangential nodes.
template <typename S, typename T>
hipError_t launch_pack(const Geom &g, int field, const S *src, T *dst, T *dst2, hipStream_t s,
                       double scale = 1.0);

// Padded box (type T) -> dense staggered buffer (type S) for field f, each value
// divided by scale in FP64.
template <typename T, typename S>
hipError_t launch_unpack(const Geom &g, int field, const T *src, S *dst, hipStream_t s, double scale = 1.0);

// Diagnostics (FP64). partial must hold diag_partial_doubles() doubles.
size_t diag_partial_doubles();
template <typename T>
hipError_t launch_diag(const Geom &g, const Fields<T> &f, const Coefs<typename Store<T>::C> &c,
                       double *partial, double *out_dev, hipStream_t s);

// How the tiled sweeps number their workgroups: 0 in plain launch order; 1 so
// each of the 8 XCDs owns one contiguous block of tiles; 2, the default
// (temporal sweeps only; the slab sweeps read it as 1), so the workgroups
// resident at one time, one per CU, cover one contiguous range of tiles, each
// XCD a contiguous part of it. FDTD_XCD_REMAP selects the mode.
int xcd_remap();

// Compute units per XCD of the current device (the device's CU count / 8).
int cus_per_xcd();

// How the temporal sweeps hand out tiles: 0 one workgroup per tile, in the
// FDTD_XCD_REMAP order; 1 (the default) one workgroup per CU taking tiles from a
// queue (the batched serving sweeps with per-node Ch: one workgroup per tile).
// FDTD_TEMPORAL_SCHED selects it.
int temporal_sched();

// Set the thread-local message fdtd_last_error returns.
void set_last_error(const char *msg);

// Staggered extents (X, Y, Z) of field f in 0..5.
__host__ __device__ inline void extents(const Geom &g, int f, int &X, int &Y, int &Z)
{
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    switch (f) {
    case 0: X = nx; Y = ny + 1; Z = nz + 1; break;
    case 1: X = nx + 1; Y = ny; Z = nz + 1; break;
    case 2: X = nx + 1; Y = ny + 1; Z = nz; break;
    case 3: X = nx + 1; Y = ny; Z = nz; break;
    case 4: X = nx; Y = ny + 1; Z = nz; break;
    default: X = nx; Y = ny; Z = nz + 1; break;
    }
}

}  // namespace fdtd
