// C ABI of libfdtd (declared and documented in include/fdtd.h).
//
// Device memory of one solver, carved from one arena (caller-provided or
// hipMalloc'd), each region 256-byte aligned:
//   A[6]  state buffer 0 (Ex Ey Ez Hx Hy Hz boxes)
//   B[6]  state buffer 1 (the fused schedules write the next state here)
//   Ce[3] per-node E coefficients (only with per-cell eps)
//   Ch[3] per-node H coefficients (only with per-cell mu)
//   staging: one dense staggered array in FP64 (host transfers, materials)
//   diag: FP64 partial sums of the diagnostics
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_set>
#include <vector>

#include "fdtd.h"
#include "fdtd_internal.h"
#include "solver.h"

namespace {
std::string &g_last_error_ref()
{
    thread_local std::string msg;
    return msg;
}
}  // namespace

namespace fdtd {
Plan make_plan(int nx, int ny, int nz, int fesz, bool ce_arr, bool ch_arr, bool aux, bool comp)
{
    auto up = [](size_t v, size_t a) { return (v + a - 1) / a * a; };
    Plan p{};
    Geom &g = p.g;
    g.nx = nx;
    g.ny = ny;
    g.nz = nz;
    g.px = (int)up((size_t)nx + 1, 64);
    g.py = ny + 1;
    g.pz = nz + 1;
    g.plane = (long long)g.px * g.py;
    g.box = (long long)up((size_t)g.plane * g.pz + 2 * kGuardElems, 64);
    p.fesz = (size_t)fesz;
    p.cesz = fesz == 8 ? 8 : 4;  // 16-bit fields keep FP32 coefficients
    // compensated storage: every box has room for a record box (kRecBytes per element, after
    // the 16-bit values); the E records use Ex's, the H records Hx's
    p.fbox_bytes = up((size_t)g.box * p.fesz, 256) + (comp ? up((size_t)g.box * kRecBytes, 256) : 0);
    g.lo_off = comp ? (long long)up((size_t)g.box * p.fesz, 256) + (long long)kGuardElems * (kRecBytes - fesz) : 0;
    g.lo_step = comp ? (long long)p.fbox_bytes - 1 : 0;
    p.cbox_bytes = up((size_t)g.box * p.cesz, 256);
    size_t off = 0;
    for (int b = 0; b < 2; ++b)
        for (int f = 0; f < 6; ++f) {
            p.off_fields[b][f] = off;
            off += p.fbox_bytes;
        }
    for (int f = 0; f < 3; ++f) {
        p.off_ce[f] = ce_arr ? off : SIZE_MAX;
        if (ce_arr) off += p.cbox_bytes;
    }
    for (int f = 0; f < 3; ++f) {
        p.off_ch[f] = ch_arr ? off : SIZE_MAX;
        if (ch_arr) off += p.cbox_bytes;
    }
    if (aux) {
        p.staging_bytes = up((size_t)(nx + 1) * (ny + 1) * (nz + 1) * sizeof(double), 256);
        p.off_staging = off;
        off += p.staging_bytes;
        p.off_diag = off;
        off += up((diag_partial_doubles() + 16) * sizeof(double), 256);
    } else {
        p.staging_bytes = 0;
        p.off_staging = p.off_diag = SIZE_MAX;
    }
    p.off_sched = off;
    off += 256;
    p.total = off;
    return p;
}

void set_last_error(const char *msg) { g_last_error_ref() = msg; }

int xcd_remap()
{
    static const int v = [] {
        const char *e = getenv("FDTD_XCD_REMAP");
        const int m = (e && *e) ? atoi(e) : 2;
        return m < 0 ? 0 : (m > 2 ? 2 : m);
    }();
    return v;
}

int temporal_sched()
{
    static const int v = [] {
        const char *e = getenv("FDTD_TEMPORAL_SCHED");
        return (e && *e) ? (atoi(e) != 0) : 1;
    }();
    return v;
}

int cus_per_xcd()
{
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        dev = 0;
    int v = cache[dev].load(std::memory_order_relaxed);
    if (v == 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 8)
            cus = 256;
        v = cus / 8;
        cache[dev].store(v, std::memory_order_relaxed);
    }
    return v;
}
}  // namespace fdtd

using fdtd::Coefs;
using fdtd::Fields;
using fdtd::Geom;

namespace {

constexpr uint32_t kMagic = 0xFD7D2025u;
constexpr uint32_t kDead = 0xDEADFD7Du;


// Live handles: a destroyed or foreign pointer is rejected without being dereferenced.
std::mutex g_live_mu;
std::unordered_set<const void *> g_live;

bool is_live(const void *h)
{
    std::lock_guard<std::mutex> lk(g_live_mu);
    return h && g_live.count(h) != 0;
}

int fail(int status, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int status, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error_ref() = buf;
    return status;
}

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

using fdtd::Plan;

bool is_comp(int storage) { return storage == FDTD_F16C || storage == FDTD_BF16C; }

Plan make_plan(int nx, int ny, int nz, int storage, bool ce_arr, bool ch_arr)
{
    return fdtd::make_plan(nx, ny, nz, storage == FDTD_F64 ? 8 : storage == FDTD_F32 ? 4 : 2, ce_arr, ch_arr, true,
                           is_comp(storage));
}

}  // namespace


namespace {

int check(fdtd_t h)
{
    if (!is_live(h) || h->magic != kMagic)
        return fail(FDTD_E_STATE, "invalid or destroyed solver handle");
    if (h->failed)
        return fail(FDTD_E_STATE, "solver is in an error state after a device failure");
    return FDTD_OK;
}

int device_fail(fdtd_t h, hipError_t e, const char *what)
{
    if (h)
        h->failed = true;
    return fail(FDTD_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Make the solver's device current for this thread.
int use_device(fdtd_t h)
{
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess)
        return device_fail(h, e, "hipSetDevice");
    return FDTD_OK;
}

template <typename T>
Fields<T> fields_of(fdtd_t h, int b)
{
    Fields<T> f;
    for (int q = 0; q < 6; ++q) f.f[q] = (T *)h->fld[b][q];
    return f;
}

// Coefficients in the compute type of storage T (FP32 for 16-bit fields).
template <typename T>
Coefs<typename fdtd::Store<T>::C> coefs_of(fdtd_t h)
{
    using C = typename fdtd::Store<T>::C;
    Coefs<C> c;
    for (int q = 0; q < 3; ++q) {
        c.ce[q] = (const C *)h->ce[q];
        c.ch[q] = (const C *)h->ch[q];
    }
    c.ce_s = (C)h->ce_s;
    c.ch_s = (C)h->ch_s;
    return c;
}

// Call fn with a value of the storage element type.
template <typename Fn>
auto by_storage(int storage, Fn &&fn)
{
    switch (storage) {
    case FDTD_F64: return fn(double{});
    case FDTD_F16: return fn(fdtd::f16{});
    case FDTD_BF16: return fn(fdtd::bf16{});
    case FDTD_F16C: return fn(fdtd::f16c{});
    case FDTD_BF16C: return fn(fdtd::bf16c{});
    default: return fn(float{});
    }
}

// 16-bit based storage (plain or compensated): built for the temporal kernel only
bool is16(int storage)
{
    return storage == FDTD_F16 || storage == FDTD_BF16 || storage == FDTD_F16C || storage == FDTD_BF16C;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int scan_material(const double *m, size_t n, double *mn, const char *name)
{
    *mn = 1.0;
    if (!m)
        return FDTD_OK;
    double lo = INFINITY;
    for (size_t q = 0; q < n; ++q) {
        if (!finite_pos(m[q]))
            return fail(FDTD_E_ARG, "%s[%zu] = %g is not finite and > 0", name, q, m[q]);
        lo = m[q] < lo ? m[q] : lo;
    }
    *mn = lo;
    return FDTD_OK;
}

// The fastest schedule measured on MI355X for each storage type: FP32 runs
// the temporal sweep (3 steps per HBM pass), FP64 the single-step slab.
int resolve_kernel(int kernel, int storage)
{
    if (kernel == FDTD_KERNEL_AUTO)
        return storage == FDTD_F64 ? FDTD_KERNEL_SLAB : FDTD_KERNEL_TEMPORAL;
    return kernel;
}

int env_int(const char *name, int dflt)
{
    const char *v = getenv(name);
    if (!v || !*v)
        return dflt;
    return atoi(v);
}

template <typename T>
hipError_t launch_one(fdtd_t h, int kernel, int ts, unsigned *queue)
{
    const auto c = coefs_of<T>(h);
    hipError_t e;
    if constexpr (sizeof(T) == 2) {
        // 16-bit storage is built for the temporal sweep only (ts = 1 for single steps)
        (void)kernel;
        e = fdtd::launch_temporal_step<T>(h->plan.g, fields_of<T>(h, h->cur), fields_of<T>(h, 1 - h->cur), c,
                                          h->tzchunk, ts, h->tvariant, h->stream, h->nt_stores, queue);
    } else {
        if (kernel == FDTD_KERNEL_PLAIN)
            return fdtd::launch_plain_step<T>(h->plan.g, fields_of<T>(h, h->cur), c, h->stream);
        if (kernel == FDTD_KERNEL_SLAB)
            e = fdtd::launch_slab_step<T>(h->plan.g, fields_of<T>(h, h->cur), fields_of<T>(h, 1 - h->cur), c,
                                          h->zchunk, h->variant, h->stream, h->nt_stores);
        else if (kernel == FDTD_KERNEL_TEMPORAL)
            e = fdtd::launch_temporal_step<T>(h->plan.g, fields_of<T>(h, h->cur), fields_of<T>(h, 1 - h->cur), c,
                                              h->tzchunk, ts, h->tvariant, h->stream, h->nt_stores, queue);
        else
            e = fdtd::launch_fused_step<T>(h->plan.g, fields_of<T>(h, h->cur), fields_of<T>(h, 1 - h->cur), c,
                                           h->zchunk, h->stream);
    }
    h->cur = 1 - h->cur;
    return e;
}

template <typename T>
int step_impl(fdtd_t h, long long n, unsigned *queue)
{
    // temporal: floor(n / tb) sweeps of tb steps, then the remainder as ONE sweep of n mod tb
    // steps (FP32: the same bits as single steps; 16-bit storage rounds the state once per
    // sweep, so a remainder sweep rounds once, as the serving pool's last round does);
    // other schedules: one launch per step
    const long long tb = h->kernel == FDTD_KERNEL_TEMPORAL ? h->tb : 1;
    const long long full = n / tb;
    const int rest = (int)(n % tb);
    for (long long s = 0; s < full; ++s) {
        hipError_t e = launch_one<T>(h, h->kernel, (int)tb, queue);
        if (e != hipSuccess)
            return device_fail(h, e, "kernel launch");
        h->steps += tb;
        h->sweeps += 1;
    }
    if (rest > 0) {
        hipError_t e = launch_one<T>(h, FDTD_KERNEL_TEMPORAL, rest, queue);
        if (e != hipSuccess)
            return device_fail(h, e, "kernel launch");
        h->steps += rest;
        h->sweeps += 1;
    }
    return FDTD_OK;
}

template <typename S, typename T>
hipError_t pack_all(fdtd_t h, const void *const src[6], bool staged)
{
    for (int f = 0; f < 6; ++f) {
        const S *p = (const S *)src[f];
        if (staged) {
            int X, Y, Z;
            fdtd::extents(h->plan.g, f, X, Y, Z);
            size_t bytes = (size_t)X * Y * Z * sizeof(S);
            hipError_t e = hipMemcpyAsync(h->staging, src[f], bytes, hipMemcpyHostToDevice, h->stream);
            if (e != hipSuccess)
                return e;
            p = (const S *)h->staging;
        }
        hipError_t e = fdtd::launch_pack<S, T>(h->plan.g, f, p, (T *)h->fld[0][f], (T *)h->fld[1][f], h->stream,
                                               h->scale[f % 3]);
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

template <typename T, typename S>
hipError_t unpack_all(fdtd_t h, void *const dst[6], bool staged, void *const *boxes, bool scaled)
{
    for (int f = 0; f < 6; ++f) {
        int X, Y, Z;
        fdtd::extents(h->plan.g, f, X, Y, Z);
        size_t bytes = (size_t)X * Y * Z * sizeof(S);
        S *out = staged ? (S *)h->staging : (S *)dst[f];
        if (!boxes[f]) {
            hipError_t e = hipMemsetAsync(out, 0, bytes, h->stream);
            if (e != hipSuccess)
                return e;
        } else {
            hipError_t e = fdtd::launch_unpack<T, S>(h->plan.g, f, (const T *)boxes[f], out, h->stream,
                                                     scaled ? h->scale[f % 3] : 1.0);
            if (e != hipSuccess)
                return e;
        }
        if (staged) {
            hipError_t e = hipMemcpyAsync(dst[f], h->staging, bytes, hipMemcpyDeviceToHost, h->stream);
            if (e != hipSuccess)
                return e;
            e = hipStreamSynchronize(h->stream);
            if (e != hipSuccess)
                return e;
        }
    }
    return hipSuccess;
}

int set_fields_common(fdtd_t h, const void *const src[6], int dtype, bool staged)
{
    int st = check(h);
    if (st)
        return st;
    if (!src)
        return fail(FDTD_E_ARG, "NULL field array");
    for (int f = 0; f < 6; ++f)
        if (!src[f])
            return fail(FDTD_E_ARG, "NULL pointer for field %d", f);
    if (dtype != FDTD_F32 && dtype != FDTD_F64)
        return fail(FDTD_E_ARG, "unsupported buffer dtype %d", dtype);
    if ((st = use_device(h)))
        return st;
    hipError_t e = by_storage(h->storage, [&](auto tag) {
        using T = decltype(tag);
        return dtype == FDTD_F32 ? pack_all<float, T>(h, src, staged) : pack_all<double, T>(h, src, staged);
    });
    if (e == hipSuccess && staged)
        e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess)
        return device_fail(h, e, "set_fields");
    h->cur = 0;
    h->steps = 0;
    h->fields_set = true;
    return FDTD_OK;
}

int get_common(fdtd_t h, void *const dst[6], int dtype, bool staged, void *const *boxes, bool coefs = false)
{
    int st = check(h);
    if (st)
        return st;
    if (!dst)
        return fail(FDTD_E_ARG, "NULL field array");
    for (int f = 0; f < 6; ++f)
        if (!dst[f])
            return fail(FDTD_E_ARG, "NULL pointer for field %d", f);
    if (dtype != FDTD_F32 && dtype != FDTD_F64)
        return fail(FDTD_E_ARG, "unsupported buffer dtype %d", dtype);
    if ((st = use_device(h)))
        return st;
    // coefficient boxes hold the compute type (FP32 for 16-bit fields)
    const int st_box = coefs ? (h->storage == FDTD_F64 ? FDTD_F64 : FDTD_F32) : h->storage;
    hipError_t e = by_storage(st_box, [&](auto tag) {
        using T = decltype(tag);
        return dtype == FDTD_F32 ? unpack_all<T, float>(h, dst, staged, boxes, !coefs)
                                 : unpack_all<T, double>(h, dst, staged, boxes, !coefs);
    });
    if (e != hipSuccess)
        return device_fail(h, e, "get_fields");
    return FDTD_OK;
}

}  // namespace

namespace fdtd {
int solver_check(fdtd_t h) { return check(h); }
int solver_device_fail(fdtd_t h, hipError_t e, const char *what) { return device_fail(h, e, what); }
int step_with_queue(fdtd_t h, long long n, unsigned *queue)
{
    int st = check(h);
    if (st)
        return st;
    if (n < 0)
        return fail(FDTD_E_ARG, "negative step count %lld", n);
    if (!h->fields_set)
        return fail(FDTD_E_STATE, "fields were never set");
    return by_storage(h->storage, [&](auto tag) { return step_impl<decltype(tag)>(h, n, queue); });
}
}  // namespace fdtd

namespace {

int device_cus(int device)
{
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1)
        cus = 256;
    return cus;
}

// z-split for a kernel whose workgroup fills a CU and takes time close to proportional to the
// planes it marches (its z-chunk plus `redo` planes): the chunk count that minimises
// (waves of workgroups over the CUs) x (planes per workgroup), chunks of >= min_planes and,
// when max_planes > 0, of at most max_planes (where nz allows).
constexpr int kTemporalMaxChunk = 384;

int best_zsplit(long long tiles, int nz, int redo, int min_planes, int cus, int max_planes = 0)
{
    long long best = -1;
    int zc_best = 1;
    for (int zc = 1; zc <= std::max(1, nz / min_planes); ++zc) {
        const long long kc = (nz + zc - 1) / zc, nzc = (nz + kc - 1) / kc;
        if (max_planes > 0 && kc > max_planes && zc < std::max(1, nz / min_planes))
            continue;
        const long long waves = (tiles * nzc + cus - 1) / cus;
        const long long cost = waves * (kc + redo);
        if (best < 0 || cost < best) {
            best = cost;
            zc_best = zc;
        }
    }
    return zc_best;
}

}  // namespace

extern "C" {

int fdtd_opts_default(fdtd_opts *o)
{
    if (!o)
        return fail(FDTD_E_ARG, "NULL opts");
    memset(o, 0, sizeof *o);
    o->storage = FDTD_F32;
    o->kernel = FDTD_KERNEL_AUTO;
    return FDTD_OK;
}

int fdtd_required_bytes(int nx, int ny, int nz, const fdtd_coef *coef, const fdtd_opts *opts, size_t *out)
{
    if (!out)
        return fail(FDTD_E_ARG, "NULL out");
    if (nx < 2 || ny < 2 || nz < 2)
        return fail(FDTD_E_ARG, "dims must be >= 2 (got %d %d %d)", nx, ny, nz);
    fdtd_opts d;
    fdtd_opts_default(&d);
    const fdtd_opts *o = opts ? opts : &d;
    if (o->storage < FDTD_F64 || o->storage > FDTD_BF16C)
        return fail(FDTD_E_UNSUPPORTED, "storage dtype %d not built", o->storage);
    const bool rect = (o->dy > 0.0 || o->dz > 0.0);  // rectangular cells keep per-node coefficient arrays
    Plan p = make_plan(nx, ny, nz, o->storage, (coef && coef->eps_r) || rect, (coef && coef->mu_r) || rect);
    *out = p.total + 256;  // room to align an arbitrary arena base
    return FDTD_OK;
}

int fdtd_create(int nx, int ny, int nz, double dx, double dt, const fdtd_coef *coef, const fdtd_opts *opts,
                fdtd_t *out)
{
    if (!out)
        return fail(FDTD_E_ARG, "NULL out");
    if (nx < 2 || ny < 2 || nz < 2)
        return fail(FDTD_E_ARG, "dims must be >= 2 (got %d %d %d)", nx, ny, nz);
    if ((long long)nx * ny * nz > (1LL << 33))
        return fail(FDTD_E_ARG, "grid too large");
    if (!finite_pos(dx) || !finite_pos(dt))
        return fail(FDTD_E_ARG, "dx and dt must be finite and > 0 (got %g, %g)", dx, dt);
    fdtd_opts d;
    fdtd_opts_default(&d);
    const fdtd_opts *o = opts ? opts : &d;
    if (o->storage < FDTD_F64 || o->storage > FDTD_BF16C)
        return fail(FDTD_E_UNSUPPORTED, "storage dtype %d not built", o->storage);
    if (o->kernel < FDTD_KERNEL_AUTO || o->kernel > FDTD_KERNEL_TEMPORAL)
        return fail(FDTD_E_ARG, "unknown kernel %d", o->kernel);
    int kern = resolve_kernel(o->kernel, o->storage);
    if (kern == FDTD_KERNEL_TEMPORAL && o->storage == FDTD_F64)
        return fail(FDTD_E_UNSUPPORTED, "the temporal kernel is not built for FP64 storage");
    if (is16(o->storage) && kern != FDTD_KERNEL_TEMPORAL)
        return fail(FDTD_E_UNSUPPORTED, "16-bit storage is built for the temporal kernel only");
    if (kern == FDTD_KERNEL_TEMPORAL && (o->tb_steps < 0 || o->tb_steps > 4))
        return fail(FDTD_E_ARG, "tb_steps must be 1..4 (0: the default), got %d", o->tb_steps);
    {
        // the sweeps address one padded x-y plane with 32-bit byte offsets and mark a dropped
        // access with an offset of 2^31, so a plane must stay below 2^31 bytes; with 16-bit
        // storage the same sweep addresses planes of FP32 coefficients and of 4-byte residual
        // records, so the bound applies to 4-byte elements there too
        const long long px = ((long long)nx + 1 + 63) / 64 * 64;
        const long long esz = o->storage == FDTD_F64 ? 8 : 4;
        if (px * (ny + 1) * esz >= (1LL << 31))
            return fail(FDTD_E_ARG, "x-y plane of %lld bytes: planes must stay below 2^31 bytes",
                        px * (ny + 1) * esz);
    }
    if (o->arena && o->arena_bytes == 0)
        return fail(FDTD_E_ARG, "arena given with arena_bytes = 0");
    if (!(o->dy == 0.0 || finite_pos(o->dy)) || !(o->dz == 0.0 || finite_pos(o->dz)))
        return fail(FDTD_E_ARG, "dy and dz must be 0 (= dx) or finite and > 0 (got %g, %g)", o->dy, o->dz);
    const double dy = o->dy > 0.0 ? o->dy : dx, dz = o->dz > 0.0 ? o->dz : dx;
    // rectangular cells (any spacing given explicitly): per-node coefficient arrays carry the
    // axis factors; a spacing equal to dx gives factor 1 and the cubic bits
    const bool rect = o->dy > 0.0 || o->dz > 0.0;
    const double *eps = coef ? coef->eps_r : nullptr;
    const double *mu = coef ? coef->mu_r : nullptr;
    const size_t ncell = (size_t)nx * ny * nz;
    double eps_min, mu_min;
    int st;
    if ((st = scan_material(eps, ncell, &eps_min, "eps_r")))
        return st;
    if ((st = scan_material(mu, ncell, &mu_min, "mu_r")))
        return st;
    // Courant limit of the Yee grid: c_max dt sqrt(1/dx^2 + 1/dy^2 + 1/dz^2) < 1,
    // c_max = 1/sqrt(min eps min mu); on cubic cells dt sqrt(3) / dx
    const double courant =
        rect ? dt * std::sqrt(1.0 / (dx * dx) + 1.0 / (dy * dy) + 1.0 / (dz * dz)) : dt * std::sqrt(3.0) / dx;
    if (!(courant < std::sqrt(eps_min * mu_min)))
        return fail(FDTD_E_CFL, "dt*sqrt(sum 1/d^2) = %.17g violates the Courant limit %.17g", courant,
                    std::sqrt(eps_min * mu_min));

    Plan p = make_plan(nx, ny, nz, o->storage, eps != nullptr || rect, mu != nullptr || rect);
    // memory limits are checked before any device call
    const size_t need = p.total + 256;
    if (o->arena && o->arena_bytes < need)
        return fail(FDTD_E_NOMEM, "arena of %zu bytes < required %zu", o->arena_bytes, need);
    if (!o->arena) {
        const char *budget = getenv("FDTD_HBM_BUDGET");
        if (budget && *budget && (double)need > atof(budget))
            return fail(FDTD_E_NOMEM, "required %zu bytes exceed FDTD_HBM_BUDGET=%s", need, budget);
    }
    hipError_t e = hipSetDevice(o->device);
    if (e != hipSuccess)
        return fail(FDTD_E_DEVICE, "hipSetDevice(%d): %s", o->device, hipGetErrorString(e));

    fdtd_solver *h = new fdtd_solver();
    h->magic = kMagic;
    h->nx = nx;
    h->ny = ny;
    h->nz = nz;
    h->dx = dx;
    h->dt = dt;
    h->d[0] = dx;
    h->d[1] = dy;
    h->d[2] = dz;
    h->scale[0] = 1.0;
    h->scale[1] = dy / dx;
    h->scale[2] = dz / dx;
    h->aniso = dy != dx || dz != dx;
    h->storage = o->storage;
    h->kernel = kern;
    h->tb = kern == FDTD_KERNEL_TEMPORAL ? (o->tb_steps > 0 ? o->tb_steps : 3) : 1;
    h->device = o->device;
    h->zchunk = env_int("FDTD_ZCHUNKS", 0);
    h->variant = env_int("FDTD_SLAB_VARIANT", 0);
    h->plan = p;
    h->ce_arr = eps != nullptr || rect;
    h->ch_arr = mu != nullptr || rect;
    h->ce_s = dt / dx;
    h->ch_s = dt / dx;
    {
        // bytes one sweep streams: both state buffers and the coefficient arrays
        const size_t streamed = 12 * p.fbox_bytes + ((h->ce_arr ? 3 : 0) + (h->ch_arr ? 3 : 0)) * p.cbox_bytes;
        h->nt_stores = streamed > fdtd::kStreamCacheBytes;
        const int force = env_int("FDTD_NT_STORES", -1);  // 0 / 1 overrides the size rule
        if (force == 0 || force == 1)
            h->nt_stores = force == 1;
    }
    const int slab_v = h->storage == FDTD_F64 ? 3 : h->variant;
    if (h->zchunk <= 0 && (kern == FDTD_KERNEL_SLAB || kern == FDTD_KERNEL_TEMPORAL) && slab_v == 0) {
        // the 16-wave slab workgroup (also the single steps of a temporal schedule) fills a CU
        // like the temporal one (see below); a z-chunk redoes one plane; chunks of >= 4 planes
        const int own = fdtd::slab_rows(0) - 2, w = fdtd::slab_width(0);
        const long long tiles = (long long)((nx + w - 1) / w) * ((ny + own - 1) / own);
        h->zchunk = best_zsplit(tiles, nz, 1, 4, device_cus(o->device));
    }
    if (h->zchunk <= 0) {
        // split z so the launch has enough workgroups to cover the 256 CUs several times
        long long tiles;
        int target;
        if (kern == FDTD_KERNEL_SLAB) {
            const int v = h->storage == FDTD_F64 ? 3 : h->variant;
            const int own = fdtd::slab_rows(v) - 2, w = fdtd::slab_width(v);
            tiles = (long long)((nx + w - 1) / w) * ((ny + own - 1) / own);
            target = fdtd::slab_rows(v) == 16 ? 1024 : 2048;
        } else {
            tiles = (long long)((nx + 63) / 64) * ((ny + 7) / 8);
            target = 2048;
        }
        int zc = 1;
        while (tiles * zc < target && nz / (zc * 2) >= 16) zc *= 2;
        h->zchunk = zc;
    }
    h->tvariant = env_int("FDTD_TEMPORAL_VARIANT", 0);
    if (kern == FDTD_KERNEL_TEMPORAL && o->tb_steps == 0)
        // default steps per sweep: 4 (512^3: FP32 258 Gcell/s against 226 at 3, 16-bit storage
        // 329-333 against 320-322, compensated 244-245 against 220-224); 3 with per-node Ch,
        // whose third coefficient pipeline spills registers at 4
        h->tb = o->storage != FDTD_F64 && !h->ch_arr && h->tvariant == 0 ? 4 : 3;
    if (h->tb > 3)
        h->tvariant = 0;  // one row per wave is built for 1..3 steps per sweep
    h->tzchunk = env_int("FDTD_TZCHUNKS", 0);
    if (h->tzchunk <= 0) {
        // One temporal workgroup per CU, and a workgroup's time is close to proportional to the
        // planes it marches (its z-chunk plus the 2*tb-1 planes it redoes): pick the split that
        // minimises waves-of-workgroups x planes per workgroup, chunks of 8 to 384 planes (the
        // tiles of one XCD drift apart over a long chunk and share fewer halo lines in L2:
        // 1024^3 ran 3 % faster in 342-plane chunks than in one 1024-plane chunk).
        const int own = fdtd::temporal_own_rows(h->tb, h->tvariant);
        const int w = fdtd::temporal_width(h->tvariant);
        const long long tiles = (long long)((nx + w - 1) / w) * ((ny + own - 1) / own);
        h->tzchunk = best_zsplit(tiles, nz, 2 * h->tb - 1, 8, device_cus(o->device), kTemporalMaxChunk);
    }
    if (o->stream) {
        h->stream = (hipStream_t)o->stream;
        h->own_stream = false;
    } else {
        e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete h;
            return fail(FDTD_E_DEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
        }
        h->own_stream = true;
    }
    char *base;
    if (o->arena) {
        h->arena = (char *)o->arena;
        h->arena_bytes = o->arena_bytes;
        h->own_arena = false;
    } else {
        void *mem = nullptr;
        e = hipMalloc(&mem, need);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            if (h->own_stream) (void)hipStreamDestroy(h->stream);
            delete h;
            return fail(FDTD_E_NOMEM, "hipMalloc(%zu): %s", need, hipGetErrorString(e));
        }
        h->arena = (char *)mem;
        h->arena_bytes = need;
        h->own_arena = true;
    }
    base = (char *)round_up((uintptr_t)h->arena, 256);
    const size_t fguard = (size_t)fdtd::kGuardElems * p.fesz, cguard = (size_t)fdtd::kGuardElems * p.cesz;
    for (int b = 0; b < 2; ++b)
        for (int f = 0; f < 6; ++f) h->fld[b][f] = base + p.off_fields[b][f] + fguard;
    for (int f = 0; f < 3; ++f) {
        h->ce[f] = h->ce_arr ? base + p.off_ce[f] + cguard : nullptr;
        h->ch[f] = h->ch_arr ? base + p.off_ch[f] + cguard : nullptr;
    }
    h->staging = base + p.off_staging;
    h->diag = (double *)(base + p.off_diag);
    h->sched = (unsigned *)(base + p.off_sched);

    e = hipMemsetAsync(base, 0, p.total, h->stream);
    // materials -> staging -> FP64 coefficient kernel, one material at a time. Rectangular
    // cells, in the stored variables E_a s_a, H_a s_a (s = 1, dy/dx, dz/dx), update like
    // cubic cells of size dx with component a's coefficient times s_a / (s_b s_c).
    const double *sc = h->scale;
    const double fac[6] = {sc[0] / (sc[1] * sc[2]), sc[1] / (sc[0] * sc[2]), sc[2] / (sc[0] * sc[1]),
                           sc[0] / (sc[1] * sc[2]), sc[1] / (sc[0] * sc[2]), sc[2] / (sc[0] * sc[1])};
    for (int which = 0; which < 2 && e == hipSuccess; ++which) {
        const double *m = which == 0 ? eps : mu;
        if (!m && !rect)
            continue;
        if (m)
            e = hipMemcpyAsync(h->staging, m, ncell * sizeof(double), hipMemcpyHostToDevice, h->stream);
        if (e != hipSuccess)
            break;
        const double *md = m ? (const double *)h->staging : nullptr;
        if (h->storage != FDTD_F64) {
            float *ce[3] = {nullptr, nullptr, nullptr}, *ch[3] = {nullptr, nullptr, nullptr};
            for (int f = 0; f < 3; ++f) (which == 0 ? ce : ch)[f] = (float *)(which == 0 ? h->ce[f] : h->ch[f]);
            e = fdtd::launch_coef<float>(p.g, dx, dt, which == 0 ? md : nullptr, which == 1 ? md : nullptr, ce, ch,
                                         h->stream, rect ? fac : nullptr);
        } else {
            double *ce[3] = {nullptr, nullptr, nullptr}, *ch[3] = {nullptr, nullptr, nullptr};
            for (int f = 0; f < 3; ++f) (which == 0 ? ce : ch)[f] = (double *)(which == 0 ? h->ce[f] : h->ch[f]);
            e = fdtd::launch_coef<double>(p.g, dx, dt, which == 0 ? md : nullptr, which == 1 ? md : nullptr, ce, ch,
                                          h->stream, rect ? fac : nullptr);
        }
        if (e == hipSuccess)
            e = hipStreamSynchronize(h->stream);  // staging is reused by the next material
    }
    if (e == hipSuccess)
        e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        int r = fail(FDTD_E_DEVICE, "create: %s", hipGetErrorString(e));
        if (h->own_arena) (void)hipFree(h->arena);
        if (h->own_stream) (void)hipStreamDestroy(h->stream);
        delete h;
        return r;
    }
    h->fields_set = false;
    {
        std::lock_guard<std::mutex> lk(g_live_mu);
        g_live.insert(h);
    }
    *out = h;
    return FDTD_OK;
}

int fdtd_set_fields(fdtd_t h, const void *const host[6], int host_dtype)
{
    return set_fields_common(h, host, host_dtype, true);
}

int fdtd_set_fields_device(fdtd_t h, const void *const dev[6], int dev_dtype)
{
    return set_fields_common(h, dev, dev_dtype, false);
}

int fdtd_init_random(fdtd_t h, unsigned long long seed)
{
    int st = check(h);
    if (st)
        return st;
    if ((st = use_device(h)))
        return st;
    hipError_t e = by_storage(h->storage, [&](auto tag) {
        using T = decltype(tag);
        T *a[6], *b[6];
        for (int f = 0; f < 6; ++f) {
            a[f] = (T *)h->fld[0][f];
            b[f] = (T *)h->fld[1][f];
        }
        return fdtd::launch_init_random<T>(h->plan.g, seed, a, b, h->stream, h->scale);
    });
    if (e != hipSuccess)
        return device_fail(h, e, "init_random");
    h->cur = 0;
    h->steps = 0;
    h->fields_set = true;
    return FDTD_OK;
}

int fdtd_step(fdtd_t h, long long n)
{
    int st = check(h);
    if (st)
        return st;
    if (n < 0)
        return fail(FDTD_E_ARG, "negative step count %lld", n);
    if (!h->fields_set)
        return fail(FDTD_E_STATE, "fields were never set");
    if ((st = use_device(h)))
        return st;
    return by_storage(h->storage, [&](auto tag) { return step_impl<decltype(tag)>(h, n, h->sched); });
}

int fdtd_get_fields(fdtd_t h, void *const host[6], int host_dtype)
{
    if (int st = check(h))
        return st;
    void *const *boxes = h->fld[h->cur];
    return get_common(h, host, host_dtype, true, boxes);
}

int fdtd_get_fields_device(fdtd_t h, void *const dev[6], int dev_dtype)
{
    if (int st = check(h))
        return st;
    void *const *boxes = h->fld[h->cur];
    return get_common(h, dev, dev_dtype, false, boxes);
}

int fdtd_get_coefs(fdtd_t h, void *const host[6], int host_dtype)
{
    if (int st = check(h))
        return st;
    if (!h->ce_arr || !h->ch_arr) {
        // scalar coefficients: materialise the per-node view the kernels apply
        // (scalar on updated nodes, 0 on nodes that never change) on the host
        if (!host)
            return fail(FDTD_E_ARG, "NULL field array");
        if (host_dtype != FDTD_F32 && host_dtype != FDTD_F64)
            return fail(FDTD_E_ARG, "unsupported buffer dtype %d", host_dtype);
    }
    void *boxes[6];
    for (int f = 0; f < 3; ++f) {
        boxes[f] = h->ce[f];
        boxes[f + 3] = h->ch[f];
    }
    int st = get_common(h, host, host_dtype, true, boxes, true);
    if (st)
        return st;
    const int nx = h->nx, ny = h->ny, nz = h->nz;
    for (int f = 0; f < 6; ++f) {
        const bool scalar = f < 3 ? !h->ce_arr : !h->ch_arr;
        if (!scalar)
            continue;
        int X, Y, Z;
        fdtd::extents(h->plan.g, f, X, Y, Z);
        const double sv = h->storage != FDTD_F64 ? (double)(float)(f < 3 ? h->ce_s : h->ch_s)
                                                 : (f < 3 ? h->ce_s : h->ch_s);
        for (int k = 0; k < Z; ++k)
            for (int j = 0; j < Y; ++j)
                for (int i = 0; i < X; ++i) {
                    bool fixed;
                    switch (f) {
                    case 0: fixed = j == 0 || j == ny || k == 0 || k == nz; break;
                    case 1: fixed = i == 0 || i == nx || k == 0 || k == nz; break;
                    case 2: fixed = i == 0 || i == nx || j == 0 || j == ny; break;
                    case 3: fixed = i == 0 || i == nx; break;
                    case 4: fixed = j == 0 || j == ny; break;
                    default: fixed = k == 0 || k == nz; break;
                    }
                    const size_t l = (size_t)i + (size_t)X * ((size_t)j + (size_t)Y * k);
                    const double v = fixed ? 0.0 : sv;
                    if (host_dtype == FDTD_F64)
                        ((double *)host[f])[l] = v;
                    else
                        ((float *)host[f])[l] = (float)v;
                }
    }
    return FDTD_OK;
}

int fdtd_sync(fdtd_t h)
{
    if (int st = check(h))
        return st;
    if (int st = use_device(h))
        return st;
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess)
        return device_fail(h, e, "sync");
    return FDTD_OK;
}

long long fdtd_steps_done(fdtd_t h)
{
    if (!is_live(h) || h->magic != kMagic)
        return -1;
    return h->steps;
}

int fdtd_diag(fdtd_t h, double out[FDTD_DIAG_N])
{
    if (int st = check(h))
        return st;
    if (!out)
        return fail(FDTD_E_ARG, "NULL out");
    if (int st = use_device(h))
        return st;
    double *partial = h->diag;
    double *dev_out = h->diag + fdtd::diag_partial_doubles();
    hipError_t e = by_storage(h->storage, [&](auto tag) {
        using T = decltype(tag);
        return fdtd::launch_diag<T>(h->plan.g, fields_of<T>(h, h->cur), coefs_of<T>(h), partial, dev_out,
                                    h->stream);
    });
    double tmp[8] = {0};
    if (e == hipSuccess)
        e = hipMemcpyAsync(tmp, dev_out, 6 * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess)
        return device_fail(h, e, "diag");
    for (int q = 0; q < FDTD_DIAG_N; ++q) out[q] = tmp[q];
    return FDTD_OK;
}

int fdtd_query(fdtd_t h, long long out[8])
{
    if (!is_live(h) || h->magic != kMagic)
        return fail(FDTD_E_STATE, "invalid or destroyed solver handle");
    if (!out)
        return fail(FDTD_E_ARG, "NULL out");
    out[0] = h->kernel;
    out[1] = h->kernel == FDTD_KERNEL_TEMPORAL ? h->tb : 1;
    out[2] = h->storage;
    out[3] = h->sweeps;
    out[4] = h->ce_arr;
    out[5] = h->ch_arr;
    out[6] = h->plan.g.px;
    out[7] = (long long)h->arena_bytes;
    return FDTD_OK;
}

void *fdtd_stream(fdtd_t h)
{
    if (!is_live(h) || h->magic != kMagic)
        return nullptr;
    return (void *)h->stream;
}

int fdtd_destroy(fdtd_t h)
{
    {
        std::lock_guard<std::mutex> lk(g_live_mu);
        if (!h || g_live.erase(h) == 0)
            return fail(FDTD_E_STATE, "invalid or destroyed solver handle");
    }
    (void)hipSetDevice(h->device);
    hipError_t e = hipStreamSynchronize(h->stream);
    if (h->own_arena)
        (void)hipFree(h->arena);
    if (h->own_stream)
        (void)hipStreamDestroy(h->stream);
    h->magic = kDead;
    delete h;
    if (e != hipSuccess)
        return fail(FDTD_E_DEVICE, "destroy: pending work failed: %s", hipGetErrorString(e));
    return FDTD_OK;
}

int fdtd_get_schedule(fdtd_t h, fdtd_schedule *out)
{
    if (!is_live(h) || h->magic != kMagic)
        return fail(FDTD_E_STATE, "invalid or destroyed solver handle");
    if (!out)
        return fail(FDTD_E_ARG, "NULL out");
    memset(out, 0, sizeof *out);
    out->kernel = h->kernel;
    out->tb_steps = h->kernel == FDTD_KERNEL_TEMPORAL ? h->tb : 1;
    out->variant = h->kernel == FDTD_KERNEL_TEMPORAL ? h->tvariant
                   : h->kernel == FDTD_KERNEL_SLAB   ? (h->storage == FDTD_F64 ? 3 : h->variant)
                                                     : 0;
    out->zchunks = h->kernel == FDTD_KERNEL_TEMPORAL ? h->tzchunk : h->kernel == FDTD_KERNEL_PLAIN ? 1 : h->zchunk;
    return FDTD_OK;
}

}  // extern "C"

namespace {

int validate_schedule(fdtd_t h, const fdtd_schedule *sc)
{
    if (sc->kernel < FDTD_KERNEL_PLAIN || sc->kernel > FDTD_KERNEL_TEMPORAL)
        return fail(FDTD_E_ARG, "unknown kernel %d", sc->kernel);
    if (is16(h->storage) && sc->kernel != FDTD_KERNEL_TEMPORAL)
        return fail(FDTD_E_UNSUPPORTED, "16-bit storage is built for the temporal kernel only");
    if (h->storage == FDTD_F64 && sc->kernel == FDTD_KERNEL_TEMPORAL)
        return fail(FDTD_E_UNSUPPORTED, "the temporal kernel is not built for FP64 storage");
    if (sc->kernel == FDTD_KERNEL_TEMPORAL && (sc->tb_steps < 1 || sc->tb_steps > 4))
        return fail(FDTD_E_ARG, "tb_steps must be 1..4, got %d", sc->tb_steps);
    if (sc->kernel == FDTD_KERNEL_TEMPORAL && (sc->variant < 0 || sc->variant > 1))
        return fail(FDTD_E_ARG, "temporal variant must be 0..1, got %d", sc->variant);
    if (sc->kernel == FDTD_KERNEL_TEMPORAL && sc->variant == 1 && sc->tb_steps > 3)
        return fail(FDTD_E_UNSUPPORTED, "temporal variant 1 is built for tb_steps 1..3");
    if (sc->kernel == FDTD_KERNEL_SLAB && (sc->variant < 0 || sc->variant > 3))
        return fail(FDTD_E_ARG, "slab variant must be 0..3, got %d", sc->variant);
    if (sc->kernel == FDTD_KERNEL_SLAB && h->storage == FDTD_F64 && sc->variant != 3)
        return fail(FDTD_E_UNSUPPORTED, "FP64 storage builds slab variant 3 only");
    if (sc->kernel != FDTD_KERNEL_PLAIN && (sc->zchunks < 1 || sc->zchunks > h->nz))
        return fail(FDTD_E_ARG, "zchunks must be 1..nz, got %d", sc->zchunks);
    return FDTD_OK;
}

void apply_schedule(fdtd_t h, const fdtd_schedule *sc)
{
    h->kernel = sc->kernel;
    if (sc->kernel == FDTD_KERNEL_TEMPORAL) {
        h->tb = sc->tb_steps;
        h->tvariant = sc->variant;
        h->tzchunk = sc->zchunks;
    } else {
        h->tb = 1;
        if (sc->kernel == FDTD_KERNEL_SLAB)
            h->variant = sc->variant;
        if (sc->kernel != FDTD_KERNEL_PLAIN)
            h->zchunk = sc->zchunks;
    }
}

std::vector<fdtd_schedule> schedule_candidates(fdtd_t h)
{
    std::vector<fdtd_schedule> out;
    std::vector<int> zcs;
    for (int zc = 1; zc <= 16; zc *= 2)
        if (zc == 1 || h->nz / zc >= 16)
            zcs.push_back(zc);
    auto add = [&](int kernel, int tb, int variant, int zc) {
        fdtd_schedule sc{};
        sc.kernel = kernel;
        sc.tb_steps = tb;
        sc.variant = variant;
        sc.zchunks = zc;
        out.push_back(sc);
    };
    if (!is16(h->storage)) {
        add(FDTD_KERNEL_PLAIN, 1, 0, 1);
        for (int zc : zcs) add(FDTD_KERNEL_FUSED, 1, 0, zc);
        for (int v = 0; v < 4; ++v) {
            if (h->storage == FDTD_F64 && v != 3)
                continue;
            for (int zc : zcs) add(FDTD_KERNEL_SLAB, 1, v, zc);
        }
    }
    // the temporal default split need not be a power of two: try it too
    std::vector<int> tzcs = zcs;
    if (std::find(tzcs.begin(), tzcs.end(), h->tzchunk) == tzcs.end())
        tzcs.push_back(h->tzchunk);
    // 16-bit storage rounds the state at the end of every sweep, so the steps per sweep set
    // the numerics: the search keeps the solver's own tb there and varies only the tiling
    const int tb_lo = is16(h->storage) ? h->tb : 1, tb_hi = is16(h->storage) ? h->tb : 4;
    if (h->storage != FDTD_F64)
        for (int tb = tb_lo; tb <= tb_hi; ++tb)
            for (int v = 0; v < 2; ++v)
                if (v == 0 || tb <= 3)
                    for (int zc : tzcs) add(FDTD_KERNEL_TEMPORAL, tb, v, zc);
    return out;
}

}  // namespace

extern "C" {

int fdtd_set_schedule(fdtd_t h, const fdtd_schedule *sc)
{
    if (int st = check(h))
        return st;
    if (!sc)
        return fail(FDTD_E_ARG, "NULL schedule");
    if (int st = validate_schedule(h, sc))
        return st;
    apply_schedule(h, sc);
    return FDTD_OK;
}

int fdtd_autotune(fdtd_t h, int trial_steps, fdtd_schedule *results, int max_results, int *n_results)
{
    if (int st = check(h))
        return st;
    if (trial_steps < 0 || max_results < 0 || (max_results > 0 && !results))
        return fail(FDTD_E_ARG, "bad autotune arguments");
    const int steps = trial_steps ? trial_steps : 6;
    if (int st = use_device(h))
        return st;
    const std::vector<fdtd_schedule> cands = schedule_candidates(h);
    // keep the state: copy the current buffer's six boxes aside
    void *backup = nullptr;
    const size_t fbox = h->plan.fbox_bytes, guard = (size_t)fdtd::kGuardElems * h->plan.fesz;
    hipError_t e = hipMalloc(&backup, 6 * fbox);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(FDTD_E_NOMEM, "autotune needs %zu bytes of scratch: %s", 6 * fbox, hipGetErrorString(e));
    }
    const int cur0 = h->cur;
    const long long steps0 = h->steps, sweeps0 = h->sweeps;
    fdtd_schedule keep;
    fdtd_get_schedule(h, &keep);
    for (int q = 0; q < 6 && e == hipSuccess; ++q)
        e = hipMemcpyAsync((char *)backup + q * fbox, (char *)h->fld[cur0][q] - guard, fbox, hipMemcpyDeviceToDevice,
                           h->stream);
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (e == hipSuccess)
        e = hipEventCreate(&ev0);
    if (e == hipSuccess)
        e = hipEventCreate(&ev1);
    int best = -1;
    double best_ms = 0;
    std::vector<double> times(cands.size(), 0.0);
    for (size_t c = 0; c < cands.size() && e == hipSuccess; ++c) {
        apply_schedule(h, &cands[c]);
        const int tb = cands[c].kernel == FDTD_KERNEL_TEMPORAL ? cands[c].tb_steps : 1;
        const long long n = (steps + tb - 1) / tb * tb;  // whole sweeps
        int st = by_storage(h->storage, [&](auto tag) { return step_impl<decltype(tag)>(h, tb, h->sched); });
        if (st == FDTD_OK && (e = hipEventRecord(ev0, h->stream)) == hipSuccess) {
            st = by_storage(h->storage, [&](auto tag) { return step_impl<decltype(tag)>(h, n, h->sched); });
            if (st == FDTD_OK)
                e = hipEventRecord(ev1, h->stream);
            if (st == FDTD_OK && e == hipSuccess)
                e = hipEventSynchronize(ev1);
        }
        if (st != FDTD_OK) {
            e = hipErrorLaunchFailure;
            break;
        }
        float ms = 0;
        if (e == hipSuccess)
            e = hipEventElapsedTime(&ms, ev0, ev1);
        times[c] = (double)ms / (double)n;
        if (best < 0 || times[c] < best_ms) {
            best = (int)c;
            best_ms = times[c];
        }
    }
    // restore the state and counters whatever happened
    h->cur = cur0;
    for (int q = 0; q < 6; ++q) {
        hipError_t e2 = hipMemcpyAsync((char *)h->fld[cur0][q] - guard, (char *)backup + q * fbox, fbox,
                                       hipMemcpyDeviceToDevice, h->stream);
        if (e == hipSuccess)
            e = e2;
    }
    hipError_t e3 = hipStreamSynchronize(h->stream);
    if (e == hipSuccess)
        e = e3;
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    (void)hipFree(backup);
    h->steps = steps0;
    h->sweeps = sweeps0;
    if (e != hipSuccess) {
        apply_schedule(h, &keep);
        return device_fail(h, e, "autotune");
    }
    apply_schedule(h, &cands[best]);
    const int nres = std::min<int>(max_results, (int)cands.size());
    for (int c = 0; c < nres; ++c) {
        results[c] = cands[c];
        results[c].ms_per_step = times[c];
    }
    if (n_results)
        *n_results = (int)cands.size();
    return FDTD_OK;
}

const char *fdtd_strerror(int status)
{
    switch (status) {
    case FDTD_OK: return "ok";
    case FDTD_E_ARG: return "invalid argument";
    case FDTD_E_CFL: return "time step violates the Courant limit";
    case FDTD_E_NOMEM: return "not enough device memory";
    case FDTD_E_DEVICE: return "device error";
    case FDTD_E_STATE: return "invalid solver state";
    case FDTD_E_UNSUPPORTED: return "unsupported option";
    case FDTD_E_TIMEOUT: return "wait timed out";
    default: return "unknown status";
    }
}

const char *fdtd_last_error(void) { return g_last_error_ref().c_str(); }

}  // extern "C"
