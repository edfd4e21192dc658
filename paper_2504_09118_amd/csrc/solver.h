// The solver handle of the C ABI, shared by the translation units that
// implement it (fdtd_api.cpp: create / step / transfers; fdtd_adjoint.cpp:
// the reverse-time gradient).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fdtd.h"
#include "fdtd_internal.h"

struct fdtd_solver {
    uint32_t magic;
    int nx, ny, nz;
    double dx, dt;
    double d[3];      // cell size along x, y, z
    double scale[3];  // stored component = physical value x scale (1, dy/dx, dz/dx)
    bool aniso;       // d[1] or d[2] differs from dx
    int storage, kernel, tb, device, zchunk, tzchunk, variant, tvariant;
    hipStream_t stream;
    bool own_stream;
    char *arena;
    size_t arena_bytes;
    bool own_arena;
    fdtd::Plan plan;
    void *fld[2][6];
    void *ce[3], *ch[3];
    bool ce_arr, ch_arr;
    bool nt_stores;  // sweeps store non-temporally (streamed bytes exceed the last-level cache)
    double ce_s, ch_s;
    void *staging;
    double *diag;
    unsigned *sched;  // scheduling counters of the temporal sweep (arena)
    int cur;
    long long steps, sweeps;
    bool failed, fields_set;
};

namespace fdtd {

// Check a handle (live, not failed); sets the thread's error message.
int solver_check(fdtd_t h);

// Mark the solver failed after a device error and set the message.
int solver_device_fail(fdtd_t h, hipError_t e, const char *what);

// fdtd_step with the temporal sweeps' scheduling counters (kSchedWords words, zero
// before and after each launch) taken from queue instead of the solver's arena.
// Same checks and errors as fdtd_step; the device must be current.
int step_with_queue(fdtd_t h, long long n, unsigned *queue);

}  // namespace fdtd
