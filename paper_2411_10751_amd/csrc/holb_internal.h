// Host-side interface between the C ABI (holb_capi.hip) and the kernel
// launchers (holb_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "holb_params.h"

namespace holb {

// One launch's worth of device pointers and parameters.
struct LaunchCtx {
    int lattice;          // 0 D2Q37, 1 D3Q39
    int storage;          // Storage
    int family;           // Family
    int variant;          // kernel variant (block order of the generic kernels)
    int frames;           // FrameMode
    KParams kp;
    const void* pop_in;   // current state (post-collision of the last step)
    void* pop_out;        // next state
    float* aux_f;         // theta field (thermal source): the one the gradient reads
    float* theta_out;     // with the previous step's gradient (grad_lag): where the step
                          // writes its own theta field for the next step; else null
    double* aux_d;        // psi field (pressure-tensor path)
    const double* tgt_in;  // wall targets read this step
    double* tgt_out;       // wall targets written this step
    double* partials;     // reduction partials
    int max_partials;     // capacity in blocks
    hipStream_t stream;
    hipEvent_t ev_begin;  // if set, recorded around the dominant kernel of a step
    hipEvent_t ev_end;
    // Walled domains: a second stream (default priority) on which a step runs
    // its wall work beside the work of `stream` that does not depend on it,
    // with the events that fork and join the two.  Null: everything on
    // `stream`.
    hipStream_t side;
    hipEvent_t ev_fork, ev_wall, ev_join;
};

int num_variants(const LaunchCtx& c);
bool variant_supported(const LaunchCtx& c, int variant);

hipError_t launch_init(const LaunchCtx& c, const float* rho, const float* u, const float* theta);
hipError_t launch_step(const LaunchCtx& c);
hipError_t launch_aux(const LaunchCtx& c);  // psi / theta field of the current state
hipError_t launch_fields(const LaunchCtx& c, float* rho, float* u, float* theta);
hipError_t launch_reduce(const LaunchCtx& c, double* out_dev);
int reduce_blocks(const LaunchCtx& c);

// Dominant kernel of one step (the one bracketed by ev_begin / ev_end): its
// name as a profiler lists it, without namespace and spaces, and the number
// of cells one launch updates.
void dominant_kernel(const LaunchCtx& c, char* name, size_t len, long long* cells);

// Offset d_i = (f^eq_i(rho, u, theta) - f^eq_i(rho, 0, theta)) / w_i of the
// 16-bit deviation storage, in the library's velocity order (host, FP64).
void deviation_reference(int lattice, double rho, const double* u, double theta, float* ref_out);

// Velocity set in library order.
int lattice_Q(int lattice);
int lattice_NS(int lattice);  // number of velocity shells
int lattice_D(int lattice);
void lattice_table(int lattice, int* c, double* w, double* c0sq);

}  // namespace holb
