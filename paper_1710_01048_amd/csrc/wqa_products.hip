// Matrix-free products y = M x and y = K x in 3D on gfx950, blocked over rows in all three
// directions (eq:LinSys with the rules of eq:GaussQuadSys and eq:GaussQuadSysStiff).
//
// With each row's weighted rule, sum_j M_ij x_j = sum_q c(x^i_q) prod_k T_k[i_k, q_k, s_k]
// x_j (j_k = i_k - p + s_k), where T_k[i, q, s] is the weight of node q of row i times
// the basis function of column i - p + s at that node (the same tables as the assembled
// matrices).  Node q of row i is grid point g = i Q + q, and every grid point is a node of
// exactly one row, so the inner sum is one tensor-product map of x to the grid,
//     u(g) = sum_j E_1[g_1, j_1] E_2[g_2, j_2] E_3[g_3, j_3] x_j,   E_k[i Q + q, i - p + s] = T_k[i, q, s],
// and y_i is the sum of c u over the row's points.  A per-row contraction (the adjoint's
// lane mapping, as in the load vector) re-derives the partial sums of x's window for
// each of the (2p+1)^2 rows around a leading pair of indices; here a work-group takes a
// block of B1 x B2 x R rows and forms each partial sum once for the whole block:
//   1. x over the block's window, (B1 + 2p) (B2 + 2p) (R + 2p) values, zero outside the
//      space, goes to LDS;
//   2. direction 3: X3[j1, j2, g3] = sum_s E_3[g3, s] x[j1, j2, s] for every window pair
//      (j1, j2) and each of the block's R Q last-direction points (lane = g3), into LDS;
//   3. direction 2 (wave w takes second-direction row i2 = b2 + w): X23[g2, j1] =
//      sum_s E_2[g2, s] X3[j1, s, g3] for the row's Q nodes g2, in registers;
//   4. direction 1, block row by block row (b1 + i1l): u(g1, g2, g3) = sum_s E_1[g1, s]
//      X23[g2, s], times the coefficient sample of the point, summed over the row's nodes
//      in q1 and q2 in registers and over q3 across the row's Q lanes.  A block row's
//      samples are all of a lane's Q^2 points of it, loaded together one block row ahead.
// Stiffness term k takes the stiffness table in direction k and the mass tables
// elsewhere, one term at a time: terms 1 and 2 read X3 of the mass table, term 3 its own
// (the same LDS buffer, refilled).  Rows at least p from both ends of a direction whose tables are
// banded (DevSpace::band) take the P + 1 entries s = q .. q + p of each node; the others
// all S.  The sums equal the per-row ones up to rounding order.
// Loads are issued in the order of their use (they complete in order): the lane's
// direction-3 table entries, the window, then the first samples, which stay in flight
// through the direction-3 phase; the work-group barriers order LDS only.
#include "wqa_internal.h"

#include <algorithm>

namespace wqa {
namespace {

template <typename T>
using uptr = const __attribute__((address_space(4))) T *;     // wave-uniform table reads

template <typename T>
__device__ __forceinline__ uptr<T> utable(const DevTabs &tb, int kind, int dir) {
    return (uptr<T>)(const T *)tb.t[kind][dir];
}

constexpr int kBlockWaves = 4;      // B2: the block's rows along direction 2, one per wave

// Work-group order.  The hardware deals work-groups round-robin over the 8 XCDs, each
// with its own L2; here each XCD takes runs of kRun consecutive blocks (the incomplete last
// run keeps the hardware's order), so that neighbouring blocks, which share the cache lines
// of their x windows and sample runs, meet in one L2.  Measured at 160^3, p = 3, on an
// earlier form of this kernel (samples loaded node q2 by node q2): runs of 8 took 0.355 /
// 0.815 ms (FP32 y = M x / y = K x) and 0.763 / 1.896 ms (FP64), against 0.367 / 0.846 and
// 0.828 / 1.938 in the hardware's order; runs of 2 and one contiguous share per XCD fell in
// between, runs of 16 (on the final form) within 2% of runs of 8.
constexpr uint32_t kRun = 8;

__device__ __forceinline__ uint32_t block_order() {
    const uint32_t b = blockIdx.x, span = 8u * kRun, full = gridDim.x / span * span;
    return b >= full ? b : b - b % span + (b % 8) * kRun + (b / 8) % kRun;
}

// Work-group barrier that orders LDS only: the global loads in flight (coefficient
// samples) stay in flight across it.  The kernel writes global memory only at its end.
// (__syncthreads() waits for every load in flight first; with it the first samples could
// not be issued ahead, and the kernel took 0.343 / 0.758 ms for FP32 y = M x / y = K x
// at 160^3 against 0.246 / 0.627.)
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <int P>
__device__ __forceinline__ bool interior(int band_bit, int64_t i, int64_t n) {
    return band_bit && i >= P && i < n - P;
}

template <typename T, int P, int B1>
struct Block {
    static constexpr int Q = P + 1, S = 2 * P + 1, R = 64 / Q, B2 = kBlockWaves;
    static constexpr int W1 = B1 + 2 * P, W2 = B2 + 2 * P, W3 = R + 2 * P;
    static constexpr int NPAIR = W1 * W2;       // window pairs (j1, j2)
    static constexpr int NX = NPAIR * W3;       // window values

    const DevSpace &sp;
    const DevTabs &tb;
    const T *xw;       // LDS window [W1][W2][W3] (written by stage_window)
    T *x3;             // LDS [NPAIR][64]
    int64_t b1, b2, b3;
    int wave, lane, i3l, q3;
    int64_t i3c;       // the lane's last-direction row, clamped into the space

    // Whether every row of the block is interior along direction 3 and its tables banded.
    __device__ __forceinline__ bool band3() const {
        return ((sp.band >> 2) & 1) && b3 >= P && b3 + R + P <= sp.n[2];
    }

    // The lane's direction-3 table entries of kind `kind`: e[s] = T_3[i3, q3, q3 + s] for
    // s <= p (banded) or T_3[i3, q3, s] for every s.  Loaded before the samples: a later
    // load would have to wait for them (loads complete in order).
    __device__ __forceinline__ void table3(int kind, bool band, T (&e)[S]) const {
        const T *tr = (const T *)tb.t[kind][2] + (i3c * Q + q3) * S;
        if (band) {
#pragma unroll
            for (int s = 0; s <= P; ++s) e[s] = tr[q3 + s];
#pragma unroll
            for (int s = P + 1; s < S; ++s) e[s] = T(0);
        } else {
#pragma unroll
            for (int s = 0; s < S; ++s) e[s] = tr[s];
        }
    }

    // Step 2: X3 for every window pair, with the lane's direction-3 table entries e.
    template <bool BAND>
    __device__ __forceinline__ void dir3(const T (&e)[S]) const {
        constexpr int NT = BAND ? P + 1 : S;
        const T *xr = xw + i3l + (BAND ? q3 : 0);
        for (int pr = wave; pr < NPAIR; pr += kBlockWaves) {
            T acc = T(0);
#pragma unroll
            for (int s = 0; s < NT; ++s) acc = fma(e[s], xr[pr * W3 + s], acc);
            x3[pr * 64 + lane] = acc;
        }
    }

    __device__ __forceinline__ void fill_x3(bool band, const T (&e)[S]) const {
        if (band) dir3<true>(e);
        else dir3<false>(e);
    }

    // Step 3 for node q2 of the wave's row i2: X[j1] = sum_s t2[q2 S + s] X3[j1, i2l + s, lane].
    template <bool BAND>
    __device__ __forceinline__ void dir2(uptr<T> t2, int q2, T (&X)[W1]) const {
        constexpr int NT = BAND ? P + 1 : S;
        const int s0 = BAND ? q2 : 0;
        const T *col = x3 + (wave + s0) * 64 + lane;
#pragma unroll
        for (int l1 = 0; l1 < W1; ++l1) {
            T acc = T(0);
#pragma unroll
            for (int s = 0; s < NT; ++s) acc = fma(t2[q2 * S + s0 + s], col[(l1 * W2 + s) * 64], acc);
            X[l1] = acc;
        }
    }

    // The coefficient samples of block row b1 + i1l in the wave's row i2 (clamped into the
    // space: i2c) at the lane's last-direction point: fv[q1][q2] (0 outside the space).  In
    // the row layout these are the lane's Q^2 values of a 4 Q^3-byte row block whose other
    // values the row's other lanes load at the same time.  Every lane loads from indices
    // clamped into the space and zeroes what lies outside afterwards: no branches, so all
    // Q^2 loads are in flight at once.
    __device__ __forceinline__ void load(const T *__restrict__ f, int i1l, int64_t i2c, bool in2,
                                         T (&fv)[Q][Q]) const {
        const int64_t n1 = sp.n[0], n2 = sp.n[1], n3 = sp.n[2];
        const int64_t i1 = b1 + i1l;
        const bool in = in2 && i1 < n1;
        const int64_t i1c = i1 < n1 ? i1 : n1 - 1;
        int64_t off, dq1, dq2;         // sample (i1, q1 = 0; i2, q2 = 0; i3, q3) and the steps
        if (sp.rows) {
            off = ((i1c * n2 + i2c) * n3 + i3c) * (Q * Q * Q) + q3;
            dq1 = Q * Q;
            dq2 = Q;
        } else {
            off = ((i1c * Q) * sp.N[1] + i2c * Q) * sp.ld + i3c * Q + q3;
            dq1 = sp.N[1] * sp.ld;
            dq2 = sp.ld;
        }
#pragma unroll
        for (int q1 = 0; q1 < Q; ++q1)
#pragma unroll
            for (int q2 = 0; q2 < Q; ++q2) {
                const T v = f[off + q1 * dq1 + q2 * dq2];
                fv[q1][q2] = in ? v : T(0);
            }
    }

    // Step 4 for block row b1 + i1l: adds sum_{q2, q1} f(g) u(g) to acc, with
    // u = sum_s t1[(i1 Q + q1) S + s] X[q2][i1l + s].
    __device__ __forceinline__ void dir1(uptr<T> t1, int i1l, const T (&fv)[Q][Q], const T (&X)[Q][W1],
                                         T &acc) const {
        const int64_t n1 = sp.n[0];
        const int64_t i1 = b1 + i1l;
        const int64_t i1c = i1 < n1 ? i1 : n1 - 1;
        if (interior<P>(sp.band & 1, i1, n1)) {
#pragma unroll
            for (int q2 = 0; q2 < Q; ++q2)
#pragma unroll
                for (int q1 = 0; q1 < Q; ++q1) {
                    const uptr<T> tr = t1 + (i1c * Q + q1) * S + q1;
                    T u = T(0);
#pragma unroll
                    for (int s = 0; s <= P; ++s) u = fma(tr[s], X[q2][i1l + q1 + s], u);
                    acc = fma(fv[q1][q2], u, acc);
                }
        } else {
#pragma unroll
            for (int q2 = 0; q2 < Q; ++q2)
#pragma unroll
                for (int q1 = 0; q1 < Q; ++q1) {
                    const uptr<T> tr = t1 + (i1c * Q + q1) * S;
                    T u = T(0);
#pragma unroll
                    for (int s = 0; s < S; ++s) u = fma(tr[s], X[q2][i1l + s], u);
                    acc = fma(fv[q1][q2], u, acc);
                }
        }
    }

    // Steps 3 and 4 of one term over the wave's row i2: direction 2 for every node q2, then
    // block row by block row direction 1 with the samples.  fv holds block row 0's samples on
    // entry (loaded by the caller ahead of the work before).  Each block row's loop loads
    // the next one's (NEXT: after the last, block row 0 of the next term's field fnext, left
    // in fv), so that they are in flight during the contraction, and every sample line is
    // used by back-to-back loads.
    template <bool NEXT>
    __device__ __forceinline__ void pass(uptr<T> t2, uptr<T> t1, const T *__restrict__ f, const T *__restrict__ fnext,
                                         bool in2, T (&fv)[Q][Q], T (&acc)[B1]) const {
        const int64_t n2 = sp.n[1];
        const int64_t i2 = b2 + wave, i2c = row2();
        const bool band2 = interior<P>((sp.band >> 1) & 1, i2, n2);
        const uptr<T> t2r = t2 + i2c * (Q * S);
        T X[Q][W1];
#pragma unroll
        for (int q2 = 0; q2 < Q; ++q2) {
            if (band2) dir2<true>(t2r, q2, X[q2]);
            else dir2<false>(t2r, q2, X[q2]);
        }
#pragma unroll
        for (int i1l = 0; i1l < B1; ++i1l) {
            T fn[Q][Q];
            if (i1l + 1 < B1) load(f, i1l + 1, i2c, in2, fn);
            else if (NEXT) load(fnext, 0, i2c, in2, fn);
            dir1(t1, i1l, fv, X, acc[i1l]);
            if (i1l + 1 < B1 || NEXT) {
#pragma unroll
                for (int q1 = 0; q1 < Q; ++q1)
#pragma unroll
                    for (int q2 = 0; q2 < Q; ++q2) fv[q1][q2] = fn[q1][q2];
            }
        }
    }

    // Step 1: the window of x, [W1][W2][W3] from (b1 - p, b2 - p, b3 - p), zero outside the
    // space, by the whole work-group (the caller synchronizes).
    __device__ __forceinline__ void stage_window(const T *__restrict__ x, T *win) const {
        // every load of the thread first, then the LDS writes: one round trip, not NIT
        const int64_t n1 = sp.n[0], n2 = sp.n[1], n3 = sp.n[2];
        constexpr int NT = 64 * kBlockWaves, NIT = (NX + NT - 1) / NT;
        T v[NIT];
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int e = wave * 64 + lane + it * NT;
            const int l3 = e % W3, pr = e / W3, l2 = pr % W2, l1 = pr / W2;
            const int64_t j1 = b1 - P + l1, j2 = b2 - P + l2, j3 = b3 - P + l3;
            v[it] = T(0);
            if (e < NX && j1 >= 0 && j1 < n1 && j2 >= 0 && j2 < n2 && j3 >= 0 && j3 < n3)
                v[it] = x[(j1 * n2 + j2) * n3 + j3];
        }
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int e = wave * 64 + lane + it * NT;
            if (e < NX) win[e] = v[it];
        }
    }

    // The wave's second-direction row, clamped into the space.
    __device__ __forceinline__ int64_t row2() const {
        const int64_t i2 = b2 + wave;
        return i2 < sp.n[1] ? i2 : sp.n[1] - 1;
    }
};

template <typename T, int P, int WHAT, int B1>
__global__ __launch_bounds__(64 * kBlockWaves) void apply_block_kernel(DevSpace sp, DevTabs tb, const T *__restrict__ cf,
                                                                      const T *__restrict__ a0,
                                                                      const T *__restrict__ a1,
                                                                      const T *__restrict__ a2,
                                                                      const T *__restrict__ x, T *__restrict__ y,
                                                                      int64_t blk0, int64_t n_blocks, int64_t nb2,
                                                                      int64_t nb3) {
    using B = Block<T, P, B1>;
    constexpr int Q = B::Q, R = B::R, S = B::S;
    __shared__ __align__(16) T xw[B::NX];
    __shared__ __align__(16) T x3[B::NPAIR * 64];
    const int64_t blk = blk0 + block_order();
    if (blk >= n_blocks) return;                                   // the whole work-group
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = (int)(threadIdx.x & 63);
    const int64_t n1 = sp.n[0], n2 = sp.n[1], n3 = sp.n[2];
    const int64_t bb3 = blk % nb3, rest = blk / nb3;
    const int64_t b1 = (rest / nb2) * B1, b2 = (rest % nb2) * kBlockWaves, b3 = bb3 * R;

    // lane = g3 - b3 Q: row b3 + i3l, node q3 (with Q = 3 the last lane has no row)
    const bool lane_row = lane < R * Q;
    const int i3l = lane_row ? lane / Q : R - 1, q3 = lane_row ? lane - (lane / Q) * Q : 0;
    const int64_t i3 = b3 + i3l;
    const bool lane_in = lane_row && i3 < n3;
    const B blk_ctx{sp, tb, xw, x3, b1, b2, b3, wave, lane, i3l, q3, i3 < n3 ? i3 : n3 - 1};
    const bool in2 = lane_in && b2 + wave < n2;

    T acc[B1];
#pragma unroll
    for (int k = 0; k < B1; ++k) acc[k] = T(0);
    // loads in order of use, since they complete in order: the direction-3 table entries,
    // the window of x, then the first term's first samples, which stay in flight while x is
    // contracted in direction 3
    const bool band3 = blk_ctx.band3();
    T e3[WHAT == kWhatM ? 1 : 2][S];
    blk_ctx.table3(0, band3, e3[0]);
    if constexpr (WHAT != kWhatM) blk_ctx.table3(1, band3, e3[WHAT == kWhatM ? 0 : 1]);
    blk_ctx.stage_window(x, xw);
    T fv[Q][Q];
    blk_ctx.load(WHAT == kWhatM ? cf : a0, 0, blk_ctx.row2(), in2, fv);
    lds_barrier();
    blk_ctx.fill_x3(band3, e3[0]);                                 // mass table in direction 3
    lds_barrier();
    if constexpr (WHAT == kWhatM) {
        blk_ctx.template pass<false>(utable<T>(tb, 0, 1), utable<T>(tb, 0, 0), cf, nullptr, in2, fv, acc);
    } else {
        // terms 1 and 2 share X3 of the mass table; term 3 refills it with the stiffness table
        blk_ctx.template pass<true>(utable<T>(tb, 0, 1), utable<T>(tb, 1, 0), a0, a1, in2, fv, acc);
        blk_ctx.template pass<true>(utable<T>(tb, 1, 1), utable<T>(tb, 0, 0), a1, a2, in2, fv, acc);
        lds_barrier();
        blk_ctx.fill_x3(band3, e3[WHAT == kWhatM ? 0 : 1]);        // stiffness table
        lds_barrier();
        blk_ctx.template pass<false>(utable<T>(tb, 0, 1), utable<T>(tb, 0, 0), a2, nullptr, in2, fv, acc);
    }

    // each row's value: the sum over its Q lanes (lanes i3l Q .. i3l Q + Q - 1)
    const int base = i3l * Q;
    const int64_t i2 = b2 + wave;
#pragma unroll
    for (int i1l = 0; i1l < B1; ++i1l) {
        T sum = acc[i1l];
#pragma unroll
        for (int k = 1; k < Q; ++k) sum += __shfl(acc[i1l], base + k, 64);
        const int64_t i1 = b1 + i1l;
        if (lane_in && lane == base && i1 < n1 && i2 < n2) y[(i1 * n2 + i2) * n3 + i3] = sum;
    }
}

// B1 (block rows along direction 1): 4.  With p = 3 a work-group holds 34 KB of LDS in FP32
// (four per CU) and 69 KB in FP64 (two per CU).  At 160^3, FP64 y = M x / y = K x took 0.48 /
// 1.22-1.25 ms with B1 = 4, 0.52-0.53 / 1.24-1.26 with 3 and 0.60-0.61 / 1.32-1.36 with 2
// (two work-groups per CU in each case: smaller blocks hide less of their load latency);
// in FP32, 2 was no faster and 3 slower.  B1 = 5 was within 3% either way in both, and 6
// or 8 in FP32 slower.
constexpr int kBlockRows1 = 4;

template <typename T, int P, int WHAT>
hipError_t run_block(const DevSpace &sp, const DevTabs &tb, const void *c, const void *const *a, const void *x,
                     void *y, hipStream_t st, int64_t max_tasks) {
    constexpr int B1 = kBlockRows1, R = 64 / (P + 1);
    const int64_t nb1 = (sp.n[0] + B1 - 1) / B1, nb2 = (sp.n[1] + kBlockWaves - 1) / kBlockWaves;
    const int64_t nb3 = (sp.n[2] + R - 1) / R;
    const int64_t blocks = nb1 * nb2 * nb3;
    // max_tasks counts waves: at most max_tasks / 4 work-groups (at least one) per dispatch
    const int64_t step = std::max<int64_t>(1, max_tasks / kBlockWaves);
    const T *a0 = nullptr, *a1 = nullptr, *a2 = nullptr;
    if (WHAT == kWhatK) {
        a0 = (const T *)a[0];
        a1 = (const T *)a[1];
        a2 = (const T *)a[2];
    }
    for (int64_t b0 = 0; b0 < blocks; b0 += step) {
        const int64_t here = std::min(step, blocks - b0);
        hipLaunchKernelGGL((apply_block_kernel<T, P, WHAT, B1>), dim3((unsigned)here), dim3(64 * kBlockWaves), 0, st,
                           sp, tb, (const T *)c, a0, a1, a2, (const T *)x, (T *)y, b0, blocks, nb2, nb3);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T, int P>
hipError_t run_block_what(int what, const DevSpace &sp, const DevTabs &tb, const void *c, const void *const *a,
                          const void *x, void *y, hipStream_t st, int64_t max_tasks) {
    if (what == kWhatM) return run_block<T, P, kWhatM>(sp, tb, c, a, x, y, st, max_tasks);
    return run_block<T, P, kWhatK>(sp, tb, c, a, x, y, st, max_tasks);
}

}  // namespace

hipError_t launch_apply_blocked(int dtype, int what, const DevSpace &sp, const DevTabs &tb, const void *c,
                                const void *const *a, const void *x, void *y, hipStream_t stream, int64_t max_tasks) {
    if (sp.d != 3 || (what != kWhatM && what != kWhatK)) return hipErrorInvalidValue;
    if (dtype == 0)
        return sp.p == 2 ? run_block_what<float, 2>(what, sp, tb, c, a, x, y, stream, max_tasks)
                         : run_block_what<float, 3>(what, sp, tb, c, a, x, y, stream, max_tasks);
    return sp.p == 2 ? run_block_what<double, 2>(what, sp, tb, c, a, x, y, stream, max_tasks)
                     : run_block_what<double, 3>(what, sp, tb, c, a, x, y, stream, max_tasks);
}

}  // namespace wqa
