// Adjoint (reverse-time) gradient of a driven-cavity probe objective with
// respect to per-cell permittivity (declared and documented in include/fdtd.h).
//
// Forward: N single leapfrog steps of the solver, each followed by the point
// source and the probe reads; the state (E^n, H^{n-1/2}) is copied to a
// checkpoint every K steps; the steps of the last segment write each H^{n+1/2}
// straight into a history slot. Backward: for each segment of K steps, last
// one first, the segment is recomputed from its checkpoint into the history
// slots (the last one is already there from the forward), then walked in
// reverse with the adjoint sweeps. With K >= N there is one segment and no
// recompute at all. Device memory: ceil(N/K) checkpoints of six boxes,
// min(K, N) history slots of three H boxes, the adjoint fields (two buffers of
// six boxes), FP64 dJ/dCe (three boxes) and the FP64 cell gradient.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <unordered_set>
#include <vector>

#include "fdtd.h"
#include "fdtd_internal.h"
#include "solver.h"

using fdtd::Coefs;
using fdtd::Fields;
using fdtd::Geom;

namespace {

constexpr uint32_t kAdjMagic = 0xFD7DAD01u;

std::mutex g_adj_mu;
std::unordered_set<const void *> g_adj;

int afail(int status, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int afail(int status, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    fdtd::set_last_error(buf);
    return status;
}

// Interior (updated) E node of component f: not tangential to a wall.
bool interior_e(const fdtd_solver *s, int f, int i, int j, int k)
{
    const int nx = s->nx, ny = s->ny, nz = s->nz;
    switch (f) {
    case 0: return i >= 0 && i < nx && j >= 1 && j < ny && k >= 1 && k < nz;
    case 1: return i >= 1 && i < nx && j >= 0 && j < ny && k >= 1 && k < nz;
    case 2: return i >= 1 && i < nx && j >= 1 && j < ny && k >= 0 && k < nz;
    default: return false;
    }
}

}  // namespace

struct fdtd_adjoint {
    uint32_t magic;
    fdtd_t s;
    int sf;
    long long so;
    std::vector<double> wave;
    int np;
    std::vector<int> pf;
    std::vector<long long> po;
    long long N;
    int K, nseg;
    int nslots;    // history slots: min(K, N)
    int hist_seg;  // the segment whose H^{n+1/2} the slots hold (-1: none)
    char *mem;
    size_t guard, fbox;
    int *d_pf;
    long long *d_po;
    double *d_rec, *d_J, *d_grad;
    char *ckpt, *hist;
    void *adj[2][6];      // two buffers of lam Ex Ey Ez, mu Hx Hy Hz (element (0,0,0) of each box)
    fdtd::ProbeList pl;   // the probes as sweep arguments (np = 0 when there are more than fit)
    double *gce[3];
    float *gpart[3];  // FP32 group sums of the gCe terms (FP32 storage), else null
    bool forward_done;
};

namespace {

int acheck(fdtd_adjoint_t a)
{
    std::lock_guard<std::mutex> lk(g_adj_mu);
    if (!a || !g_adj.count(a) || a->magic != kAdjMagic)
        return afail(FDTD_E_STATE, "invalid or destroyed adjoint handle");
    return FDTD_OK;
}

// Start of the box that holds element (0,0,0) at p.
char *box_of(const fdtd_adjoint *a, void *p) { return (char *)p - a->guard; }

template <typename T>
Fields<T> state_of(fdtd_t s)
{
    Fields<T> f;
    for (int q = 0; q < 6; ++q) f.f[q] = (T *)s->fld[s->cur][q];
    return f;
}

template <typename T>
Fields<T> other_of(fdtd_t s)
{
    Fields<T> f;
    for (int q = 0; q < 6; ++q) f.f[q] = (T *)s->fld[1 - s->cur][q];
    return f;
}

template <typename T>
Coefs<T> coefs_of(fdtd_t s)
{
    Coefs<T> c;
    for (int q = 0; q < 3; ++q) {
        c.ce[q] = (const T *)s->ce[q];
        c.ch[q] = (const T *)s->ch[q];
    }
    c.ce_s = (T)s->ce_s;
    c.ch_s = (T)s->ch_s;
    return c;
}

// Point source of step n and the probe list as extras of one slab sweep.
fdtd::SlabExtras extras_of(const fdtd_adjoint *a, long long n, double *rec_row)
{
    fdtd::SlabExtras x{};
    const long long P = a->s->plan.g.plane;
    x.sf = a->sf;
    x.sk = a->sf >= 0 ? (int)(a->so / P) : 0;
    x.sxy = a->sf >= 0 ? (int)(a->so % P) : 0;
    x.w = a->sf >= 0 ? a->wave[n] : 0.0;
    x.pl = a->pl;
    x.rec_row = rec_row && a->pl.np > 0 ? rec_row : nullptr;
    return x;
}

// One driven step: one slab sweep of the solver that also adds the point source to its E node
// and records the probes (rec_row null: none; with more probes than a sweep carries, a probe
// kernel records them); J is summed from the records after the forward.
template <typename T>
T *hist_slot(const fdtd_adjoint *a, long long q, int f)
{
    return (T *)(a->hist + ((size_t)q * 3 + f) * a->fbox + a->guard);
}

// One driven step. h_src / h_dst, when not null, replace the solver's H buffers as the
// step's H input / output (the history slots); E always goes from the solver's current
// buffer to the other one.
template <typename T>
int driven_step(fdtd_adjoint_t a, long long n, double *rec_row, T *const *h_src = nullptr, T *const *h_dst = nullptr)
{
    fdtd_t s = a->s;
    const fdtd::SlabExtras x = extras_of(a, n, rec_row);
    Fields<T> src = state_of<T>(s), dst = other_of<T>(s);
    for (int f = 0; f < 3; ++f) {
        if (h_src)
            src.f[3 + f] = h_src[f];
        if (h_dst)
            dst.f[3 + f] = h_dst[f];
    }
    hipError_t e = fdtd::launch_slab_step<T>(s->plan.g, src, dst, coefs_of<T>(s), s->zchunk, s->variant, s->stream,
                                             s->nt_stores, &x);
    if (e != hipSuccess)
        return fdtd::solver_device_fail(s, e, "driven sweep");
    s->cur = 1 - s->cur;
    s->steps += 1;
    s->sweeps += 1;
    if (rec_row && a->np > 0 && a->pl.np == 0) {
        // the probe kernel reads E only; it also sums J, here into a spare word (J comes from the
        // records)
        e = fdtd::launch_source_probe<T>(state_of<T>(s), -1, 0, 0.0, a->np, a->d_pf, a->d_po, rec_row, a->d_J + 1,
                                         s->stream);
        if (e != hipSuccess)
            return fdtd::solver_device_fail(s, e, "probe kernel");
    }
    return FDTD_OK;
}

hipError_t copy_state(fdtd_adjoint_t a, char *dst, bool to_solver)
{
    fdtd_t s = a->s;
    for (int q = 0; q < 6; ++q) {
        char *box = box_of(a, s->fld[s->cur][q]);
        char *slot = dst + (size_t)q * a->fbox;
        hipError_t e = to_solver ? hipMemcpyAsync(box, slot, a->fbox, hipMemcpyDeviceToDevice, s->stream)
                                 : hipMemcpyAsync(slot, box, a->fbox, hipMemcpyDeviceToDevice, s->stream);
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

template <typename T>
int forward_impl(fdtd_adjoint_t a, double *J)
{
    fdtd_t s = a->s;
    hipError_t e = hipMemsetAsync(a->d_J, 0, sizeof(double), s->stream);
    if (e == hipSuccess)
        e = hipMemsetAsync(a->d_rec, 0, (size_t)(a->N + 1) * a->np * sizeof(double), s->stream);
    if (e != hipSuccess)
        return fdtd::solver_device_fail(s, e, "adjoint forward");
    // The last segment writes each H^{n+1/2} into its history slot (the backward's recompute
    // of that segment would write the same bits there); its last step runs a second time with
    // the solver's buffer as the H output, so the solver ends in state N like any forward.
    a->hist_seg = -1;
    const long long nl = (long long)(a->nseg - 1) * a->K;
    for (long long n = 0; n < a->N; ++n) {
        if (n % a->K == 0 && (e = copy_state(a, a->ckpt + (size_t)(n / a->K) * 6 * a->fbox, false)) != hipSuccess)
            return fdtd::solver_device_fail(s, e, "checkpoint");
        double *rec = a->d_rec + (size_t)(n + 1) * a->np;
        if (n < nl) {
            if (int st = driven_step<T>(a, n, rec))
                return st;
            continue;
        }
        T *hin[3], *hout[3];
        for (int f = 0; f < 3; ++f) {
            hin[f] = n > nl ? hist_slot<T>(a, n - nl - 1, f) : nullptr;
            hout[f] = hist_slot<T>(a, n - nl, f);
        }
        if (int st = driven_step<T>(a, n, rec, n > nl ? hin : nullptr, hout))
            return st;
        if (n == a->N - 1) {
            s->cur = 1 - s->cur;  // back to the step's input state
            s->steps -= 1;
            s->sweeps -= 1;
            if (int st = driven_step<T>(a, n, rec, n > nl ? hin : nullptr))
                return st;
        }
    }
    a->hist_seg = a->nseg - 1;
    if (a->np > 0 && (e = fdtd::launch_probe_objective(a->d_rec, a->N, a->np, a->d_J, s->stream)) != hipSuccess)
        return fdtd::solver_device_fail(s, e, "probe objective");
    double hJ = 0.0;
    e = hipMemcpyAsync(&hJ, a->d_J, sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess)
        return fdtd::solver_device_fail(s, e, "adjoint forward");
    *J = hJ;
    a->forward_done = true;
    return FDTD_OK;
}

template <typename T>
int backward_impl(fdtd_adjoint_t a, double *grad, void *const lam0[3], int lam0_dtype)
{
    fdtd_t s = a->s;
    const Geom &g = s->plan.g;
    Fields<T> adj;
    const Coefs<T> c = coefs_of<T>(s);
    // the fused reverse sweep (default) reads one adjoint buffer and writes the other; the plain
    // form (FDTD_ADJ_FUSED=0: one-cell-per-thread mu and lam kernels plus the probe kernel) works
    // in place on buffer 0; both give the same bits
    const char *fe = getenv("FDTD_ADJ_FUSED");
    const bool fused = !(fe && fe[0] == '0');
    int cur = 0;
    auto adj_of = [&](int b) {
        Fields<T> f;
        for (int q = 0; q < 6; ++q) f.f[q] = (T *)a->adj[b][q];
        return f;
    };
    adj = adj_of(0);
    hipError_t e = hipSuccess;
    for (int b = 0; b < 2; ++b)
        for (int q = 0; q < 6 && e == hipSuccess; ++q)
            e = hipMemsetAsync(box_of(a, a->adj[b][q]), 0, a->fbox, s->stream);
    for (int q = 0; q < 3 && e == hipSuccess; ++q)
        e = hipMemsetAsync((char *)a->gce[q] - fdtd::kGuardElems * sizeof(double), 0,
                           (size_t)g.box * sizeof(double), s->stream);
    for (int q = 0; q < 3 && a->gpart[0] && e == hipSuccess; ++q)
        e = hipMemsetAsync((char *)a->gpart[q] - fdtd::kGuardElems * sizeof(float), 0,
                           (size_t)g.box * sizeof(float), s->stream);
    if (e == hipSuccess)
        e = fdtd::launch_adj_probe<T>(adj, a->np, a->d_pf, a->d_po, a->d_rec + (size_t)a->N * a->np, s->stream);
    if (e != hipSuccess)
        return fdtd::solver_device_fail(s, e, "adjoint setup");
    // The recompute writes each H^{n+1/2} straight into its history slot: single steps of the
    // slab sweep (the bits of every schedule) with the slot as the H output and the solver's
    // two E buffers alternating. A sweep writes every H node that any sweep reads (the cells it
    // leaves alone, past the walls and in the padding, are read by no stencil), so the slots
    // need no other set-up; they were cleared once at creation, which keeps those cells finite.
    auto slot_h = [&](long long q, int f) { return hist_slot<T>(a, q, f); };
    for (int seg = a->nseg - 1; seg >= 0; --seg) {
        const long long n0 = (long long)seg * a->K, n1 = std::min(a->N, n0 + a->K);
        const bool held = seg == a->hist_seg;  // the forward (or the last recompute) left it there
        if (!held) {
            a->hist_seg = -1;
            if ((e = copy_state(a, a->ckpt + (size_t)seg * 6 * a->fbox, true)) != hipSuccess)
                return fdtd::solver_device_fail(s, e, "restore checkpoint");
        }
        for (long long n = held ? n1 : n0; n < n1; ++n) {
            const long long q = n - n0;
            const int ein = (int)(q & 1) ? 1 - s->cur : s->cur;
            Fields<T> src, dst;
            for (int f = 0; f < 3; ++f) {
                src.f[f] = (T *)s->fld[ein][f];
                dst.f[f] = (T *)s->fld[1 - ein][f];
                src.f[3 + f] = q == 0 ? (T *)s->fld[s->cur][3 + f] : slot_h(q - 1, f);
                dst.f[3 + f] = slot_h(q, f);
            }
            const fdtd::SlabExtras x = extras_of(a, n, nullptr);
            e = fdtd::launch_slab_step<T>(g, src, dst, c, s->zchunk, s->variant, s->stream, s->nt_stores, &x);
            if (e != hipSuccess)
                return fdtd::solver_device_fail(s, e, "recompute step");
        }
        a->hist_seg = seg;
        for (long long n = n1 - 1; n >= n0; --n) {
            const T *h[3];
            for (int f = 0; f < 3; ++f) h[f] = slot_h(n - n0, f);
            // the step n with n % kAdjGroup == 0 closes its group (n = 0 closes the last)
            if (fused) {
                const double *rec = n >= 1 ? a->d_rec + (size_t)n * a->np : nullptr;
                e = fdtd::launch_adj_sweep<T>(g, adj_of(cur), adj_of(1 - cur), c, h, a->gce,
                                              a->gpart[0] ? a->gpart : nullptr, n % fdtd::kAdjGroup == 0, a->pl,
                                              rec, s->zchunk, s->stream);
                cur = 1 - cur;
                if (e == hipSuccess && rec && a->np > 0 && a->pl.np == 0)
                    e = fdtd::launch_adj_probe<T>(adj_of(cur), a->np, a->d_pf, a->d_po, rec, s->stream);
            } else {
                e = fdtd::launch_adj_step<T>(g, adj, c, h, a->gce, a->gpart[0] ? a->gpart : nullptr,
                                             n % fdtd::kAdjGroup == 0, s->stream);
                if (e == hipSuccess && n >= 1)
                    e = fdtd::launch_adj_probe<T>(adj, a->np, a->d_pf, a->d_po, a->d_rec + (size_t)n * a->np,
                                                  s->stream);
            }
            if (e != hipSuccess)
                return fdtd::solver_device_fail(s, e, "adjoint step");
        }
    }
    // the solver leaves with the forward's starting state (the recompute used its buffers)
    e = copy_state(a, a->ckpt, true);
    if (e == hipSuccess)
        e = fdtd::launch_grad_eps<T>(g, c, a->gce, s->dx / s->dt, a->d_grad, s->stream);
    const size_t ncell = (size_t)s->nx * s->ny * s->nz;
    if (e == hipSuccess)
        e = hipMemcpyAsync(grad, a->d_grad, ncell * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    for (int q = 0; q < 3 && lam0 && e == hipSuccess; ++q) {
        int X, Y, Z;
        fdtd::extents(g, q, X, Y, Z);
        const size_t n = (size_t)X * Y * Z;
        if (lam0_dtype == FDTD_F64) {
            e = fdtd::launch_unpack<T, double>(g, q, (const T *)a->adj[cur][q], (double *)s->staging, s->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(lam0[q], s->staging, n * sizeof(double), hipMemcpyDeviceToHost, s->stream);
        } else {
            e = fdtd::launch_unpack<T, float>(g, q, (const T *)a->adj[cur][q], (float *)s->staging, s->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(lam0[q], s->staging, n * sizeof(float), hipMemcpyDeviceToHost, s->stream);
        }
        if (e == hipSuccess)
            e = hipStreamSynchronize(s->stream);  // staging is reused by the next component
    }
    if (e == hipSuccess)
        e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess)
        return fdtd::solver_device_fail(s, e, "adjoint gradient");
    return FDTD_OK;
}

}  // namespace

extern "C" {

int fdtd_adjoint_create(fdtd_t s, const fdtd_adjoint_problem *p, fdtd_adjoint_t *out)
{
    if (int st = fdtd::solver_check(s))
        return st;
    if (!p || !out)
        return afail(FDTD_E_ARG, "NULL argument");
    if (s->storage != FDTD_F32 && s->storage != FDTD_F64)
        return afail(FDTD_E_UNSUPPORTED, "the adjoint is built for FP32 and FP64 storage");
    if (!s->ce_arr)
        return afail(FDTD_E_UNSUPPORTED, "the permittivity gradient needs a solver created with per-cell eps_r");
    if (s->aniso)
        return afail(FDTD_E_UNSUPPORTED, "the adjoint is built for cubic cells");
    if (p->nsteps < 1)
        return afail(FDTD_E_ARG, "nsteps must be >= 1 (got %lld)", p->nsteps);
    if (p->checkpoint_every < 0)
        return afail(FDTD_E_ARG, "checkpoint_every must be >= 0 (got %d)", p->checkpoint_every);
    if (p->src_field >= 0) {
        if (!interior_e(s, p->src_field, p->src_i, p->src_j, p->src_k))
            return afail(FDTD_E_ARG, "source (%d: %d %d %d) is not an interior E node", p->src_field, p->src_i,
                         p->src_j, p->src_k);
        if (!p->waveform)
            return afail(FDTD_E_ARG, "NULL waveform");
        for (long long n = 0; n < p->nsteps; ++n)
            if (!std::isfinite(p->waveform[n]))
                return afail(FDTD_E_ARG, "waveform[%lld] is not finite", n);
    }
    if (p->nprobes < 0 || (p->nprobes > 0 && !p->probes))
        return afail(FDTD_E_ARG, "bad probe list");
    if (p->nprobes > 4096)
        return afail(FDTD_E_ARG, "at most 4096 probes (got %d)", p->nprobes);
    for (int q = 0; q < p->nprobes; ++q) {
        const int *pr = p->probes + 4 * q;
        if (!interior_e(s, pr[0], pr[1], pr[2], pr[3]))
            return afail(FDTD_E_ARG, "probe %d (%d: %d %d %d) is not an interior E node", q, pr[0], pr[1], pr[2],
                         pr[3]);
    }
    hipError_t e = hipSetDevice(s->device);
    if (e != hipSuccess)
        return afail(FDTD_E_DEVICE, "hipSetDevice: %s", hipGetErrorString(e));

    fdtd_adjoint *a = new fdtd_adjoint();
    a->magic = kAdjMagic;
    a->s = s;
    const Geom &g = s->plan.g;
    a->sf = p->src_field >= 0 ? p->src_field : -1;
    a->so = a->sf >= 0 ? g.at(p->src_i, p->src_j, p->src_k) : 0;
    if (a->sf >= 0)
        a->wave.assign(p->waveform, p->waveform + p->nsteps);
    a->np = p->nprobes;
    for (int q = 0; q < p->nprobes; ++q) {
        const int *pr = p->probes + 4 * q;
        a->pf.push_back(pr[0]);
        a->po.push_back(g.at(pr[1], pr[2], pr[3]));
    }
    a->N = p->nsteps;
    a->guard = (size_t)fdtd::kGuardElems * s->plan.fesz;
    a->fbox = s->plan.fbox_bytes;
    // checkpoints and history for interval k: ceil(N/k) states and min(k, N) H-fields
    auto stored = [&](long long k) {
        return (size_t)((a->N + k - 1) / k) * 6 * a->fbox + (size_t)std::min(k, a->N) * 3 * a->fbox;
    };
    long long K = p->checkpoint_every;
    if (K == 0) {
        // automatic: the whole history (no recompute) when it takes at most half of the free
        // device memory (and fits FDTD_HBM_BUDGET when set), else the interval that needs the
        // least memory, about sqrt(2N)
        size_t fr = 0, tot = 0;
        double cap = hipMemGetInfo(&fr, &tot) == hipSuccess ? 0.5 * (double)fr : 0.0;
        const char *budget = getenv("FDTD_HBM_BUDGET");
        if (budget && *budget)
            cap = std::min(cap, atof(budget));
        K = (double)stored(a->N) <= cap ? a->N : std::max(1LL, (long long)std::ceil(std::sqrt(2.0 * (double)a->N)));
    }
    K = std::min(K, a->N);
    a->K = (int)K;
    a->nseg = (int)((a->N + K - 1) / K);
    a->nslots = (int)K;
    a->hist_seg = -1;
    const size_t gbox = ((size_t)g.box * sizeof(double) + 255) / 256 * 256;
    const size_t ncell = (size_t)s->nx * s->ny * s->nz;
    auto up = [](size_t v) { return (v + 255) / 256 * 256; };
    size_t off = 0;
    const size_t o_ckpt = off;
    off += (size_t)a->nseg * 6 * a->fbox;
    const size_t o_hist = off;
    off += (size_t)a->nslots * 3 * a->fbox;
    const size_t o_adj = off;
    off += 12 * a->fbox;
    const size_t o_gce = off;
    off += 3 * gbox;
    // FP32 storage: the per-step gCe terms are summed in FP32 over groups of kAdjGroup steps
    const bool grouped = s->storage == FDTD_F32;
    const size_t pbox = ((size_t)g.box * sizeof(float) + 255) / 256 * 256;
    const size_t o_gpart = off;
    if (grouped)
        off += 3 * pbox;
    const size_t o_grad = off;
    off += up(ncell * sizeof(double));
    const size_t o_rec = off;
    off += up((size_t)(a->N + 1) * std::max(1, a->np) * sizeof(double));
    const size_t o_j = off;
    off += 256;
    const size_t o_pf = off;
    off += up((size_t)std::max(1, a->np) * sizeof(int));
    const size_t o_po = off;
    off += up((size_t)std::max(1, a->np) * sizeof(long long));

    e = hipMalloc((void **)&a->mem, off);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete a;
        return afail(FDTD_E_NOMEM, "adjoint needs %zu device bytes: %s", off, hipGetErrorString(e));
    }
    a->ckpt = a->mem + o_ckpt;
    a->hist = a->mem + o_hist;
    for (int b = 0; b < 2; ++b)
        for (int q = 0; q < 6; ++q) a->adj[b][q] = a->mem + o_adj + (size_t)(6 * b + q) * a->fbox + a->guard;
    for (int q = 0; q < 3; ++q)
        a->gce[q] = (double *)(a->mem + o_gce + (size_t)q * gbox) + fdtd::kGuardElems;
    for (int q = 0; q < 3; ++q)
        a->gpart[q] = grouped ? (float *)(a->mem + o_gpart + (size_t)q * pbox) + fdtd::kGuardElems : nullptr;
    a->d_grad = (double *)(a->mem + o_grad);
    a->d_rec = (double *)(a->mem + o_rec);
    a->d_J = (double *)(a->mem + o_j);
    a->d_pf = (int *)(a->mem + o_pf);
    a->d_po = (long long *)(a->mem + o_po);
    a->pl = fdtd::ProbeList{};
    if (a->np <= fdtd::kInlineProbes) {
        a->pl.np = a->np;
        for (int q = 0; q < a->np; ++q) {
            a->pl.pf[q] = a->pf[q];
            a->pl.pk[q] = (int)(a->po[q] / g.plane);
            a->pl.pxy[q] = (int)(a->po[q] % g.plane);
        }
    }
    // history slots cleared once: the cells no sweep writes stay finite (no stencil reads them)
    e = hipMemsetAsync(a->hist, 0, (size_t)a->nslots * 3 * a->fbox, s->stream);
    if (a->np && e == hipSuccess) {
        e = hipMemcpyAsync(a->d_pf, a->pf.data(), a->np * sizeof(int), hipMemcpyHostToDevice, s->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(a->d_po, a->po.data(), a->np * sizeof(long long), hipMemcpyHostToDevice, s->stream);
    }
    if (e == hipSuccess)
        e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        (void)hipFree(a->mem);
        delete a;
        return afail(FDTD_E_DEVICE, "adjoint setup: %s", hipGetErrorString(e));
    }
    {
        std::lock_guard<std::mutex> lk(g_adj_mu);
        g_adj.insert(a);
    }
    *out = a;
    return FDTD_OK;
}

int fdtd_adjoint_forward(fdtd_adjoint_t a, double *J)
{
    if (int st = acheck(a))
        return st;
    if (int st = fdtd::solver_check(a->s))
        return st;
    if (!J)
        return afail(FDTD_E_ARG, "NULL J");
    if (!a->s->fields_set)
        return afail(FDTD_E_STATE, "fields were never set");
    if (hipSetDevice(a->s->device) != hipSuccess)
        return afail(FDTD_E_DEVICE, "hipSetDevice failed");
    a->forward_done = false;
    return a->s->storage == FDTD_F64 ? forward_impl<double>(a, J) : forward_impl<float>(a, J);
}

int fdtd_adjoint_backward(fdtd_adjoint_t a, double *grad_eps, void *const lam0[3], int lam0_dtype)
{
    if (int st = acheck(a))
        return st;
    if (int st = fdtd::solver_check(a->s))
        return st;
    if (!grad_eps)
        return afail(FDTD_E_ARG, "NULL grad_eps");
    if (lam0 && (!lam0[0] || !lam0[1] || !lam0[2]))
        return afail(FDTD_E_ARG, "NULL pointer in lam0");
    if (lam0 && lam0_dtype != FDTD_F32 && lam0_dtype != FDTD_F64)
        return afail(FDTD_E_ARG, "unsupported lam0 dtype %d", lam0_dtype);
    if (!a->forward_done)
        return afail(FDTD_E_STATE, "backward needs a completed forward");
    if (hipSetDevice(a->s->device) != hipSuccess)
        return afail(FDTD_E_DEVICE, "hipSetDevice failed");
    return a->s->storage == FDTD_F64 ? backward_impl<double>(a, grad_eps, lam0, lam0_dtype)
                                     : backward_impl<float>(a, grad_eps, lam0, lam0_dtype);
}

int fdtd_adjoint_destroy(fdtd_adjoint_t a)
{
    {
        std::lock_guard<std::mutex> lk(g_adj_mu);
        if (!a || g_adj.erase(a) == 0)
            return afail(FDTD_E_STATE, "invalid or destroyed adjoint handle");
    }
    hipError_t e = hipSuccess;
    if (a->mem) {
        // the solver's stream may still read the buffers
        if (fdtd::solver_check(a->s) == FDTD_OK)
            e = hipStreamSynchronize(a->s->stream);
        else
            e = hipDeviceSynchronize();
        (void)hipFree(a->mem);
    }
    a->magic = 0;
    delete a;
    if (e != hipSuccess)
        return afail(FDTD_E_DEVICE, "adjoint destroy: %s", hipGetErrorString(e));
    return FDTD_OK;
}

}  // extern "C"
