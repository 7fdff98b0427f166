// Internal interface between the host library (wqa_host.cpp) and the HIP kernels
// (wqa_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wqa {

constexpr int kMaxDim = 3;

enum What { kWhatM = 1, kWhatK = 2, kWhatMK = 3 };

// Sizes of the tensor-product space as the kernels see them.
struct DevSpace {
    int d, p;
    int band;             // bit k: every row at least p from both ends of direction k has
                          // tables (both kinds) that vanish outside q <= s <= q + p
    int64_t n[kMaxDim];   // basis functions per direction
    int64_t N[kMaxDim];   // grid points per direction (n * (p + 1))
    int64_t ld;           // values between consecutive grid lines of the last direction (>= N[d-1])
    int rows;             // 1: samples stored row by row ([rows][Q^d]); 0: on the grid
};

// Largest number of wave tasks one kernel dispatch takes by default; larger launches
// are split into several dispatches (HIP's grid size is counted in work-items, 32 bits).
constexpr int64_t kMaxTasksPerDispatch = int64_t(1) << 24;

// Contraction tables T[kind][dir] laid out [n_dir][Q][S] on the device, in the call's
// dtype, plus FP64 copies for the FP64-accumulated final pass.
struct DevTabs {
    const void *t[2][kMaxDim];
    const double *t64[2][kMaxDim];
};

// Forward assembly (mass, stiffness or both).  dtype 0 = FP32, 1 = FP64.
// max_tasks: wave tasks per dispatch (launches with more are split).
hipError_t launch_forward(int dtype, int final_mode, int what, const DevSpace &sp,
                          const DevTabs &tb, const void *c, const void *const *a,
                          void *M, void *K, hipStream_t stream, int64_t max_tasks);

// Adjoint (either or both upstream gradients).
hipError_t launch_adjoint(int dtype, int final_mode, int what, const DevSpace &sp,
                          const DevTabs &tb, const void *gM, const void *gK,
                          void *dc, void *const *da, hipStream_t stream, int64_t max_tasks);

// Matrix-free product y = M x (what = kWhatM, coefficient c) or y = K x (kWhatK,
// coefficients a) in 2D, or with ones = true the load vector y_i = integral c B_i (x unused)
// in 2D and 3D; 3D products return hipErrorInvalidValue (they run launch_apply_blocked).
hipError_t launch_apply(int dtype, int what, bool ones, const DevSpace &sp, const DevTabs &tb,
                        const void *c, const void *const *a, const void *x, void *y, hipStream_t stream,
                        int64_t max_tasks);

// The same products in 3D (not the load vector), blocked over rows in every direction
// (wqa_products.hip); what = kWhatM or kWhatK, sp.d = 3.
hipError_t launch_apply_blocked(int dtype, int what, const DevSpace &sp, const DevTabs &tb, const void *c,
                                const void *const *a, const void *x, void *y, hipStream_t stream,
                                int64_t max_tasks);

}  // namespace wqa
