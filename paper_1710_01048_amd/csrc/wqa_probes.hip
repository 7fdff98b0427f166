// Memory-pattern probes for libwqa's kernels (libwqa_probes.so; see include/wqa_probes.h).
//
// Each probe reproduces the address stream of one kernel -- its tiles, work-group order,
// load and store instructions and the points in the stream where it stores -- but does
// no arithmetic beyond touching the loaded data, so its time is the memory system's
// price for that layout alone.  The work-group orders are restated here (the XCD
// remaps of the kernels: the hardware deals work-groups round-robin over 8 XCDs).
#include "wqa_probes.h"

#include <hip/hip_runtime.h>

#include <algorithm>

namespace {

struct Grid3 {
    int64_t n[3];   // basis functions per direction
    int64_t N[3];   // grid points per direction
    int64_t pitch;  // distance of consecutive grid lines of the outputs (N[2] unless padded)
    int rowpts;     // samples stored row by row ([rows][(p+1)^3]) instead of on the grid
};

Grid3 grid_of(int p, const int64_t *n_elem) {
    Grid3 g;
    for (int k = 0; k < 3; ++k) {
        g.n[k] = n_elem[k] + p;
        g.N[k] = g.n[k] * (p + 1);
    }
    g.pitch = g.N[2];
    g.rowpts = 0;
    return g;
}

// each XCD one contiguous share of the work-groups (the adjoint's order)
__device__ __forceinline__ uint32_t order_chunked() {
    const uint32_t b = blockIdx.x, nb = gridDim.x, q = nb / 8, r = nb % 8, x = b % 8, i = b / 8;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// runs of 8 consecutive work-groups per XCD (the forward's order)
__device__ __forceinline__ uint32_t order_grouped8() {
    const uint32_t b = blockIdx.x, span = 64u, full = gridDim.x / span * span;
    if (b >= full) return b;
    return b - b % span + (b % 8) * 8 + (b / 8) % 8;
}

// runs of 128 consecutive work-groups per XCD (the forward's order with samples by row)
__device__ __forceinline__ uint32_t order_grouped128() {
    const uint32_t b = blockIdx.x, span = 1024u, full = gridDim.x / span * span;
    if (b >= full) return b;
    return b - b % span + (b % 8) * 128 + (b / 8) % 128;
}

// 0: each XCD a contiguous share, 1: dispatch order, 2: runs of 8 per XCD
__device__ __forceinline__ uint32_t order_of(int order) {
    return order == 0 ? order_chunked() : order == 1 ? blockIdx.x : order_grouped8();
}

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void glb_void_t;

// ---- streaming ------------------------------------------------------------------------
using f4 = float __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void stream_kernel(int what, f4 *__restrict__ dst, const f4 *__restrict__ src,
                                                     int64_t n16) {
    // each wave moves 4 consecutive kilobytes per step (four 16-byte accesses per lane in
    // flight), consecutive waves consecutive 4 KB blocks
    const int64_t waves = (int64_t)gridDim.x * 4;
    const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int64_t base = wave * 256; base < n16; base += waves * 256) {
        if (base + 256 <= n16) {
            if (what == 0) {
#pragma unroll
                for (int u = 0; u < 4; ++u) dst[base + 64 * u + lane] = f4{1.f, 2.f, 3.f, 4.f};
            } else if (what == 1) {
                f4 v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) v[u] = src[base + 64 * u + lane];
#pragma unroll
                for (int u = 0; u < 4; ++u) acc += v[u];
            } else {
                f4 v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) v[u] = src[base + 64 * u + lane];
#pragma unroll
                for (int u = 0; u < 4; ++u) dst[base + 64 * u + lane] = v[u];
            }
        } else {
            for (int64_t i = base + lane; i < n16; i += 64) {
                if (what == 0) dst[i] = f4{1.f, 2.f, 3.f, 4.f};
                else if (what == 1) acc += src[i];
                else dst[i] = src[i];
            }
        }
    }
    if (what == 1 && acc.x == 1234.5f && acc.y == -1.f) dst[0] = acc;   // never true for real data
}

// k write fronts: front f covers [f * spacing, f * spacing + per_front) bytes of dst; wave
// w writes 4 KB blocks of front w % k, consecutive waves of one front consecutive blocks
__global__ __launch_bounds__(256) void fronts_kernel(char *__restrict__ dst, int k, int64_t spacing, int64_t per_front) {
    const int64_t waves = (int64_t)gridDim.x * 4;
    const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t blocks_per_front = per_front / 4096;
    for (int64_t b = wave; b < blocks_per_front * k; b += waves) {
        const int64_t f = b % k, i = b / k;
        f4 *p = reinterpret_cast<f4 *>(dst + f * spacing + i * 4096);
#pragma unroll
        for (int u = 0; u < 4; ++u) p[64 * u + lane] = f4{1.f, 2.f, 3.f, 4.f};
    }
}

// ---- the adjoint's pattern --------------------------------------------------------------
template <int N>
__device__ __forceinline__ void wait_vm() {
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

template <typename T, int P, int RING_ = 0>
struct AdjShape {
    static constexpr int Q = P + 1, S = 2 * P + 1, SL = S * S, SD = S * SL;
    static constexpr int R = 64 / Q;                    // rows per wave tile
    static constexpr int U = (int)sizeof(T) / 4;        // dwords per value
    static constexpr int NE = R * SL * U;               // dwords of one slab
    static constexpr int NPF = (NE + 63) / 64;          // loads per lane per slab
    static constexpr int SLOT = 64 * NPF;
    static constexpr int RING = RING_ ? RING_ : (sizeof(T) == 4 ? 4 : 3);
};

template <typename T, int P, int PARTS, bool DEFER = false, int RING_ = 0>
__global__ __launch_bounds__(64) void adjoint_tile_probe(Grid3 g, const T *__restrict__ gM, const T *__restrict__ gK,
                                                         T *__restrict__ o0, T *__restrict__ o1, T *__restrict__ o2,
                                                         T *__restrict__ o3, int64_t n_tasks, int tiles_per_line,
                                                         int order) {
    using A = AdjShape<T, P, RING_>;
    constexpr int Q = A::Q, S = A::S, SL = A::SL, SD = A::SD, R = A::R, U = A::U, NE = A::NE, NPF = A::NPF;
    constexpr int SLOT = A::SLOT, RING = A::RING;
    __shared__ __align__(16) uint32_t ring[RING * SLOT];
    const int lane = threadIdx.x;
    const int64_t task = order_of(order);
    if (task >= n_tasks) return;
    const int64_t line = task / tiles_per_line;
    const int tile = (int)(task - line * tiles_per_line);
    const int64_t i1 = line / g.n[1], i2 = line - i1 * g.n[1];
    const int64_t t0 = (int64_t)tile * R;
    const int rows_here = (int)std::min<int64_t>(R, g.n[2] - t0);
    const int64_t row0 = line * g.n[2] + t0;
    const bool active = lane / Q < rows_here;
    uint32_t goff[NPF];
#pragma unroll
    for (int k = 0; k < NPF; ++k) {
        const int dw = lane + 64 * k, e = dw / U, half = dw - e * U, rr = e / SL, tt = e - rr * SL;
        goff[k] = (dw < NE && rr < rows_here) ? (uint32_t)((rr * SD + tt) * U + half) : 0u;
    }
    const int s1_lo = i1 >= P ? 0 : (int)(P - i1);
    const int s1_hi = (int)std::min<int64_t>(S - 1, g.n[0] - 1 - i1 + P);
    const int ns = s1_hi - s1_lo + 1, n_tot = 2 * ns;
    auto issue = [&](int pos) {
        const T *src = pos < ns ? gM : gK;
        const int s1 = s1_lo + (pos < ns ? pos : pos - ns);
        const uint32_t *base = reinterpret_cast<const uint32_t *>(src + (row0 * SD + (int64_t)s1 * SL));
        uint32_t *dst = ring + (pos % RING) * SLOT;
#pragma unroll
        for (int k = 0; k < NPF; ++k)
            __builtin_amdgcn_global_load_lds((glb_void_t *)(base + goff[k]), (lds_void_t *)(dst + 64 * k), 4, 0, 0);
    };
    const int64_t N1 = g.N[1], N2 = g.N[2];
    const uint32_t lo = (uint32_t)(t0 * Q + lane);
    T acc = T(0);
    auto emit = [&](int run, int q1) {
        T *outs[3] = {run == 0 ? o0 : o1, o2, o3};
        const int nset = run == 0 ? 1 : 3;
        if (g.rowpts == 3) {
            // row by row, after each matrix's last slab, straight from the lanes: one
            // 4-byte store per lane and (q1, q2), (p+1) values per row and store
            if (q1 != Q - 1 || !active) return;
            const int r = lane / Q, q3 = lane - r * Q;
            for (int m = 0; m < nset; ++m)
                for (int a1 = 0; a1 < Q; ++a1)
#pragma unroll
                    for (int q2 = 0; q2 < Q; ++q2)
                        outs[m][(row0 + r) * Q * Q * Q + (a1 * Q + q2) * Q + q3] = acc + T(q2);
            return;
        }
        if (g.rowpts == 2) {
            // row by row, each q1 as it completes: the 4 lanes of a row hold its (p+1)^2
            // values of that q1 (after a transpose within the quad), one 16-byte store each
            // (p = 3: 64 bytes per row, 256 bytes apart)
            if (!active) return;
            using V4 = T __attribute__((ext_vector_type(4)));
            const int r = lane / Q, j = lane - r * Q;
            for (int m = 0; m < nset; ++m)
                *reinterpret_cast<V4 *>(outs[m] + (row0 + r) * Q * Q * Q + q1 * Q * Q + j * Q) = V4{acc, acc, acc, acc};
            return;
        }
        if (g.rowpts == 5) {
            // line-q1 blocks ([i1][i2][q1][i3][q2][q3], p = 3): as each q1 completes, the
            // tile's (i3, q2, q3) values of that q1 are one contiguous 1 KB block, written
            // with one 16-byte store per lane (lane (r, j): q2 = j, q3 = 0..3 after a
            // transpose within its quad)
            if (!active) return;
            using V4 = T __attribute__((ext_vector_type(4)));
            const int64_t line = row0 / g.n[2];
            for (int m = 0; m < nset; ++m)
                *reinterpret_cast<V4 *>(outs[m] + ((line * Q + q1) * g.n[2] + t0) * Q * Q + lane * 4) =
                    V4{acc, acc, acc, acc + T(q1)};
            return;
        }
        if (g.rowpts == 4) {
            // the same blocks after each matrix's last slab, in the order a lane (r, q_3)
            // would hold them after a transpose within its quad: one 16-byte store per q1,
            // the (p+1)^2 values of row r with q2 = j (64 bytes per row and store)
            if (q1 != Q - 1 || !active) return;
            using V4 = T __attribute__((ext_vector_type(4)));
            const int r = lane / Q, j = lane - r * Q;
            for (int m = 0; m < nset; ++m)
#pragma unroll
                for (int a1 = 0; a1 < Q; ++a1)
                    *reinterpret_cast<V4 *>(outs[m] + (row0 + r) * Q * Q * Q + (a1 * Q + j) * Q) =
                        V4{acc, acc, acc, acc + T(a1)};
            return;
        }
        if (g.rowpts) {
            // the tile's rows of each field are one contiguous block of rows_here (p+1)^3
            // values: written with 16-byte stores once per matrix run
            if (q1 != Q - 1) return;
            using V4 = T __attribute__((ext_vector_type(4)));
            const int nvec = rows_here * Q * Q * Q / 4;
            for (int m = 0; m < nset; ++m) {
                V4 *dst = reinterpret_cast<V4 *>(outs[m] + row0 * Q * Q * Q);
                for (int k = lane; k < nvec; k += 64) dst[k] = V4{acc, acc, acc, acc};
            }
            return;
        }
        if (!active) return;
        for (int m = 0; m < nset; ++m)
#pragma unroll
            for (int q2 = 0; q2 < Q; ++q2)
                (outs[m] + ((i1 * Q + q1) * N1 + i2 * Q + q2) * g.pitch)[lo] = acc + T(q2);
    };
    (void)N2;
    if constexpr (PARTS & 1)
        for (int pos = 0; pos < RING - 1 && pos < n_tot; ++pos) issue(pos);
    for (int pos = 0; pos < n_tot; ++pos) {
        const int run = pos < ns ? 0 : 1;
        const int s1 = s1_lo + (run == 0 ? pos : pos - ns);
        if constexpr (PARTS & 1) {
            asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
            if (pos + RING - 1 < n_tot) issue(pos + RING - 1);
            wait_vm<0>();
            const uint32_t v = ring[(pos % RING) * SLOT + lane];
            acc += (T)(v & 1u);
        }
        if constexpr (PARTS & 2) {
            if (DEFER) {
                if (s1 == s1_hi)
                    for (int q1 = 0; q1 < Q; ++q1) emit(run, q1);
            } else {
                if (s1 >= P) emit(run, s1 - P);
                if (s1 == s1_hi)
                    for (int q1 = s1_hi - P + 1; q1 < Q; ++q1) emit(run, q1);
            }
        }
    }
    if constexpr (!(PARTS & 2)) {
        if (acc == T(-12345)) o0[lane] = acc;   // keeps the loads (never true)
    }
}

// Line blocks: a work-group of W waves takes W consecutive tiles of one line (a whole line
// when it has at most W tiles); the waves stream their slabs in step, and after slab
// s_1 >= p the gradients of node q_1 = s_1 - p go through LDS, so that the work-group
// writes each (field, q_1) as runs of whole segments -- for a whole line one contiguous
// chunk of (p+1) grid lines -- with 16-byte stores.
template <typename T, int P, int PARTS, int RING>
__global__ __launch_bounds__(1024) void adjoint_block_probe(Grid3 g, const T *__restrict__ gM, const T *__restrict__ gK,
                                                            T *__restrict__ o0, T *__restrict__ o1,
                                                            T *__restrict__ o2, T *__restrict__ o3, int64_t n_blocks,
                                                            int tiles_per_line, int seg_tiles, int segs_per_line,
                                                            int order) {
    using A = AdjShape<T, P>;
    constexpr int Q = A::Q, S = A::S, SL = A::SL, SD = A::SD, R = A::R, U = A::U, NE = A::NE, NPF = A::NPF;
    constexpr int SLOT = A::SLOT, VEC = 16 / (int)sizeof(T);
    using VO = T __attribute__((ext_vector_type(VEC)));
    extern __shared__ __align__(16) uint32_t smem[];
    const int W = (int)(blockDim.x >> 6);
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = (int)(threadIdx.x & 63);
    const int64_t blk = order_of(order);
    if (blk >= n_blocks) return;                        // uniform over the work-group
    const int64_t line = blk / segs_per_line;
    const int seg = (int)(blk - line * segs_per_line);
    const int64_t i1 = line / g.n[1], i2 = line - i1 * g.n[1];
    const int tile = seg * seg_tiles + wave;
    const bool tile_ok = tile < tiles_per_line;
    const int64_t t0 = (int64_t)tile * R;
    const int rows_here = tile_ok ? (int)std::min<int64_t>(R, g.n[2] - t0) : 0;
    const int64_t row0 = line * g.n[2] + t0;
    const int64_t seg_t0 = (int64_t)seg * seg_tiles * R;
    const int seg_pts = (int)std::min<int64_t>((int64_t)seg_tiles * R, g.n[2] - seg_t0) * Q;
    const bool whole = segs_per_line == 1;             // the Q grid lines of a (field, q1) are one chunk
    // staged values per (field, q2): a whole line's Q grid lines are staged back to back,
    // like their global layout
    const int stride = whole ? (int)g.N[2] : seg_tiles * R * Q;
    uint32_t *ring = smem + wave * RING * SLOT;
    T *stage = reinterpret_cast<T *>(smem + W * RING * SLOT);
    uint32_t goff[NPF];
#pragma unroll
    for (int k = 0; k < NPF; ++k) {
        const int dw = lane + 64 * k, e = dw / U, half = dw - e * U, rr = e / SL, tt = e - rr * SL;
        goff[k] = (dw < NE && rr < rows_here) ? (uint32_t)((rr * SD + tt) * U + half) : 0u;
    }
    const int s1_lo = i1 >= P ? 0 : (int)(P - i1);
    const int s1_hi = (int)std::min<int64_t>(S - 1, g.n[0] - 1 - i1 + P);
    const int ns = s1_hi - s1_lo + 1, n_tot = 2 * ns;
    auto issue = [&](int pos) {
        if (!tile_ok) return;
        const T *src = pos < ns ? gM : gK;
        const int s1 = s1_lo + (pos < ns ? pos : pos - ns);
        const uint32_t *base = reinterpret_cast<const uint32_t *>(src + (row0 * SD + (int64_t)s1 * SL));
        uint32_t *dst = ring + (pos % RING) * SLOT;
#pragma unroll
        for (int k = 0; k < NPF; ++k)
            __builtin_amdgcn_global_load_lds((glb_void_t *)(base + goff[k]), (lds_void_t *)(dst + 64 * k), 4, 0, 0);
    };
    const int64_t N1 = g.N[1], N2 = g.N[2];
    T acc = T(0);
    auto emit = [&](int run, int q1) {
        T *outs[3] = {run == 0 ? o0 : o1, o2, o3};
        const int nset = run == 0 ? 1 : 3;
        if (lane < rows_here * Q)
            for (int m = 0; m < nset; ++m)
#pragma unroll
                for (int q2 = 0; q2 < Q; ++q2) stage[(m * Q + q2) * stride + wave * R * Q + lane] = acc + T(q2);
        __syncthreads();
        for (int m = 0; m < nset; ++m) {
            const int nrun = whole ? 1 : Q;
            const int len = whole ? Q * seg_pts : seg_pts;
            for (int r = 0; r < nrun; ++r) {
                T *dst = outs[m] + ((i1 * Q + q1) * N1 + i2 * Q + r) * N2 + seg_t0 * Q;
                const T *src = stage + (m * Q + r) * stride;
                const int head = (int)((VEC - (((uintptr_t)dst / sizeof(T)) & (VEC - 1))) & (VEC - 1));
                const int h = head < len ? head : len;
                for (int e = (int)threadIdx.x; e < h; e += (int)blockDim.x) dst[e] = src[e];
                const int nvec = (len - h) / VEC;
                const bool lds_aligned = (((uintptr_t)(src + h)) & 15) == 0;
                for (int k = (int)threadIdx.x; k < nvec; k += (int)blockDim.x) {
                    VO v;
                    const int e = h + k * VEC;
                    if (lds_aligned) {
                        v = *reinterpret_cast<const VO *>(src + e);
                    } else {
#pragma unroll
                        for (int c = 0; c < VEC; ++c) v[c] = src[e + c];
                    }
                    *reinterpret_cast<VO *>(dst + e) = v;
                }
                for (int e = h + nvec * VEC + (int)threadIdx.x; e < len; e += (int)blockDim.x) dst[e] = src[e];
            }
        }
        __syncthreads();
    };
    if constexpr (PARTS & 1)
        for (int pos = 0; pos < RING - 1 && pos < n_tot; ++pos) issue(pos);
    for (int pos = 0; pos < n_tot; ++pos) {
        const int run = pos < ns ? 0 : 1;
        const int s1 = s1_lo + (run == 0 ? pos : pos - ns);
        if constexpr (PARTS & 1) {
            asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
            if (pos + RING - 1 < n_tot) issue(pos + RING - 1);
            wait_vm<0>();
            const uint32_t v = ring[(pos % RING) * SLOT + lane];
            acc += (T)(v & 1u);
        }
        if constexpr (PARTS & 2) {
            if (s1 >= P) emit(run, s1 - P);
            if (s1 == s1_hi)
                for (int q1 = s1_hi - P + 1; q1 < Q; ++q1) emit(run, q1);
        }
    }
    if constexpr (!(PARTS & 2)) {
        if (acc == T(-12345)) o0[lane] = acc;   // keeps the loads (never true)
    }
}

template <typename T, int P, int PARTS, int RING>
int launch_adjoint_block(const Grid3 &g, int max_tiles, const void *gM, const void *gK, void *const *out,
                         hipStream_t st, int order) {
    using A = AdjShape<T, P>;
    const int tiles = (int)((g.n[2] + A::R - 1) / A::R);
    const int segs = (tiles + max_tiles - 1) / max_tiles;
    const int seg_tiles = (tiles + segs - 1) / segs;
    const int64_t blocks = g.n[0] * g.n[1] * segs;
    const size_t lds = (size_t)seg_tiles * RING * A::SLOT * 4 +
                       ((PARTS & 2) ? (size_t)3 * A::Q * seg_tiles * A::R * A::Q * sizeof(T) : 0);
    if (lds > 160 * 1024 || seg_tiles > 16 || blocks >= (int64_t(1) << 26)) return -1;
    if (hipFuncSetAttribute((const void *)adjoint_block_probe<T, P, PARTS, RING>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return -5;
    hipLaunchKernelGGL((adjoint_block_probe<T, P, PARTS, RING>), dim3((unsigned)blocks), dim3(64 * seg_tiles), lds, st,
                       g, (const T *)gM, (const T *)gK, (T *)out[0], (T *)out[1], (T *)out[2], (T *)out[3], blocks,
                       tiles, seg_tiles, segs, order);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

// Bulk: per wave tile, each matrix's rows of the tile (one contiguous range) are loaded
// into LDS at once with direct global-to-LDS loads, then the tile's gradients of that
// matrix are written (q_1 by q_1), then the next matrix.
template <typename T, int P, int PARTS>
__global__ __launch_bounds__(64) void adjoint_bulk_probe(Grid3 g, const T *__restrict__ gM, const T *__restrict__ gK,
                                                         T *__restrict__ o0, T *__restrict__ o1, T *__restrict__ o2,
                                                         T *__restrict__ o3, int64_t n_tasks, int tiles_per_line,
                                                         int order) {
    using A = AdjShape<T, P>;
    constexpr int Q = A::Q, SD = A::SD, R = A::R, U = A::U;
    constexpr int NDW = R * SD * U;                     // dwords of one matrix's tile rows
    constexpr int NL = (NDW + 63) / 64;
    __shared__ __align__(16) uint32_t buf[NL * 64];
    const int lane = threadIdx.x;
    const int64_t task = order_of(order);
    if (task >= n_tasks) return;
    const int64_t line = task / tiles_per_line;
    const int tile = (int)(task - line * tiles_per_line);
    const int64_t i1 = line / g.n[1], i2 = line - i1 * g.n[1];
    const int64_t t0 = (int64_t)tile * R;
    const int rows_here = (int)std::min<int64_t>(R, g.n[2] - t0);
    const int64_t row0 = line * g.n[2] + t0;
    const bool active = lane / Q < rows_here;
    const int ndw = rows_here * SD * U;
    const int64_t N1 = g.N[1], N2 = g.N[2];
    const uint32_t lo = (uint32_t)(t0 * Q + lane);
    T acc = T(0);
    for (int run = 0; run < 2; ++run) {
        if constexpr (PARTS & 1) {
            const uint32_t *src = reinterpret_cast<const uint32_t *>((run == 0 ? gM : gK) + row0 * SD);
            for (int k = 0; k < NL; ++k) {
                const int dw = 64 * k + lane;
                __builtin_amdgcn_global_load_lds((glb_void_t *)(src + (dw < ndw ? dw : 0)), (lds_void_t *)(buf + 64 * k),
                                                 4, 0, 0);
            }
            wait_vm<0>();
            acc += (T)(buf[lane] & 1u);
            __builtin_amdgcn_wave_barrier();
        }
        if constexpr (PARTS & 2) {
            if (active) {
                T *outs[3] = {run == 0 ? o0 : o1, o2, o3};
                const int nset = run == 0 ? 1 : 3;
                for (int q1 = 0; q1 < Q; ++q1)
                    for (int m = 0; m < nset; ++m)
#pragma unroll
                        for (int q2 = 0; q2 < Q; ++q2)
                            (outs[m] + ((i1 * Q + q1) * N1 + i2 * Q + q2) * N2)[lo] = acc + T(q2);
            }
        }
    }
    if constexpr (!(PARTS & 2)) {
        if (acc == T(-12345)) o0[lane] = acc;   // keeps the loads (never true)
    }
}

template <typename T, int P, int PARTS>
int launch_adjoint_bulk(const Grid3 &g, const void *gM, const void *gK, void *const *out, hipStream_t st,
                        int order) {
    constexpr int R = AdjShape<T, P>::R;
    const int tiles = (int)((g.n[2] + R - 1) / R);
    const int64_t tasks = g.n[0] * g.n[1] * tiles;
    if (tasks >= (int64_t(1) << 31) / 64) return -1;
    hipLaunchKernelGGL((adjoint_bulk_probe<T, P, PARTS>), dim3((unsigned)tasks), dim3(64), 0, st, g,
                       (const T *)gM, (const T *)gK, (T *)out[0], (T *)out[1], (T *)out[2], (T *)out[3], tasks,
                       tiles, order);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

template <typename T, int P, int PARTS, bool DEFER = false, int RING_ = 0>
int launch_adjoint_tile(const Grid3 &g, const void *gM, const void *gK, void *const *out, hipStream_t st,
                        int order, int cap8 = 0) {
    constexpr int R = AdjShape<T, P>::R;
    const int tiles = (int)((g.n[2] + R - 1) / R);
    const int64_t tasks = g.n[0] * g.n[1] * tiles;
    if (tasks >= (int64_t(1) << 31) / 64) return -1;
    // cap8: dynamic LDS that brings each work-group to 20 KB, so that at most 8 share a CU
    using A = AdjShape<T, P, RING_>;
    constexpr int kStatic = A::RING * A::SLOT * 4;
    const size_t dyn = (cap8 && kStatic < 20480) ? (size_t)(20480 - kStatic) : 0;
    hipLaunchKernelGGL((adjoint_tile_probe<T, P, PARTS, DEFER, RING_>), dim3((unsigned)tasks), dim3(64), dyn, st, g,
                       (const T *)gM, (const T *)gK, (T *)out[0], (T *)out[1], (T *)out[2], (T *)out[3], tasks,
                       tiles, order);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

template <typename T, int P, int RING>
int adjoint_block_parts(int parts, int max_tiles, const Grid3 &g, const void *gM, const void *gK, void *const *out,
                        hipStream_t st, int order) {
    switch (parts) {
        case 1: return launch_adjoint_block<T, P, 1, RING>(g, max_tiles, gM, gK, out, st, order);
        case 2: return launch_adjoint_block<T, P, 2, RING>(g, max_tiles, gM, gK, out, st, order);
        case 3: return launch_adjoint_block<T, P, 3, RING>(g, max_tiles, gM, gK, out, st, order);
        default: return -1;
    }
}

// layout 0: the kernel's tiles; layout = 16 r + t (t >= 1): line blocks of at most t
// tiles with a ring of r + 2 slabs per wave (r in 0..2)
template <typename T, int P>
int adjoint_parts(int parts, int layout, const Grid3 &g, const void *gM, const void *gK, void *const *out,
                  hipStream_t st) {
    const int order = (layout >> 6) & 3;    // 0: each XCD a contiguous share, 1: dispatch, 2: runs of 8
    Grid3 gp = g;
    if (layout & 256) gp.pitch = (g.N[2] + 31) / 32 * 32;   // output lines start 128-byte aligned (FP32)
    if (layout & 512) gp.rowpts = 1;                         // gradients stored row by row
    if (layout & 1024) gp.rowpts = 2;                        // ... each q1 as it completes (p = 3)
    if (layout & 2048) gp.rowpts = 3;                        // ... after the run, 4-byte stores
    const bool ring3 = (layout & 4096) != 0;                 // a ring of 3 slabs (more waves per CU)
    const int cap8 = (layout & 8192) ? 1 : 0;                // at most 8 waves per CU
    if (layout & 16384) gp.rowpts = 4;                       // row blocks in the lanes' order
    if (layout & 32768) gp.rowpts = 5;                       // line-q1 blocks as each q1 completes
    layout &= 63;
    if (layout == 0 && (ring3 || cap8 || gp.pitch != g.N[2] || gp.rowpts)) {
        if (ring3) {
            switch (parts) {
                case 2: return launch_adjoint_tile<T, P, 2, false, 3>(gp, gM, gK, out, st, order);
                case 3: return launch_adjoint_tile<T, P, 3, false, 3>(gp, gM, gK, out, st, order);
                default: return -1;
            }
        }
        switch (parts) {
            case 2: return launch_adjoint_tile<T, P, 2>(gp, gM, gK, out, st, order, cap8);
            case 3: return launch_adjoint_tile<T, P, 3>(gp, gM, gK, out, st, order, cap8);
            default: return -1;
        }
    }
    if (layout == 48) {
        switch (parts) {
            case 1: return launch_adjoint_bulk<T, P, 1>(g, gM, gK, out, st, order);
            case 2: return launch_adjoint_bulk<T, P, 2>(g, gM, gK, out, st, order);
            case 3: return launch_adjoint_bulk<T, P, 3>(g, gM, gK, out, st, order);
            default: return -1;
        }
    }
    if (layout == 49) {
        switch (parts) {
            case 2: return launch_adjoint_tile<T, P, 2, true>(g, gM, gK, out, st, order);
            case 3: return launch_adjoint_tile<T, P, 3, true>(g, gM, gK, out, st, order);
            default: return -1;
        }
    }
    if (layout > 0) {
        const int t = layout % 16, r = layout / 16;
        if (t < 1) return -1;
        switch (r) {
            case 0: return adjoint_block_parts<T, P, 2>(parts, t, g, gM, gK, out, st, order);
            case 1: return adjoint_block_parts<T, P, 3>(parts, t, g, gM, gK, out, st, order);
            case 2: return adjoint_block_parts<T, P, 4>(parts, t, g, gM, gK, out, st, order);
            default: return -1;
        }
    }
    switch (parts) {
        case 1: return launch_adjoint_tile<T, P, 1>(g, gM, gK, out, st, order);
        case 2: return launch_adjoint_tile<T, P, 2>(g, gM, gK, out, st, order);
        case 3: return launch_adjoint_tile<T, P, 3>(g, gM, gK, out, st, order);
        default: return -1;
    }
}

// ---- the forward's pattern --------------------------------------------------------------
template <typename T, int P, int PARTS, int ORDER>
__global__ __launch_bounds__(64) void forward_probe(Grid3 g, const T *__restrict__ f0, const T *__restrict__ f1,
                                                    const T *__restrict__ f2, const T *__restrict__ f3,
                                                    T *__restrict__ Mo, T *__restrict__ Ko, int64_t n_tasks,
                                                    int tiles_per_line, int flags) {
    constexpr int Q = P + 1, S = 2 * P + 1, SD = S * S * S, R = 64 / S, NG = Q * Q, NF = 4;
    constexpr int U = (Q * (int)sizeof(T)) % 16 == 0 ? 16 / (int)sizeof(T) : 1;
    constexpr int PER = R * Q / U, TOT = NG * PER, IT = (TOT + 63) / 64;
    constexpr int VEC = 16 / (int)sizeof(T);
    constexpr int OUT = R * SD + VEC, IN = NF * NG * R * Q;
    using VT = T __attribute__((ext_vector_type(U)));
    using VO = T __attribute__((ext_vector_type(VEC)));
    __shared__ __align__(16) T stage[OUT > IN ? OUT : IN];
    const int lane = threadIdx.x;
    const int64_t task = ORDER == 0 ? order_grouped8() : ORDER == 1 ? order_chunked() : ORDER == 3 ? order_grouped128()
                                                                                                 : blockIdx.x;
    if (task >= n_tasks) return;
    const int64_t line = task / tiles_per_line;
    const int tile = (int)(task - line * tiles_per_line);
    const int64_t i1 = line / g.n[1], i2 = line - i1 * g.n[1];
    const int64_t t0 = (int64_t)tile * R;
    const int rows_here = (int)std::min<int64_t>(R, g.n[2] - t0);
    const int64_t row0 = line * g.n[2] + t0;
    if ((PARTS & 1) && g.rowpts) {
        // the tile's rows of each field: one contiguous block of rows_here (p+1)^3 samples
        using V4 = T __attribute__((ext_vector_type(4)));
        constexpr int QD = Q * Q * Q, NV = (R * QD / 4 + 63) / 64;
        const int nvec = rows_here * QD / 4;
        const T *fl[NF] = {f0, f1, f2, f3};
        V4 v[NF][NV];
#pragma unroll
        for (int m = 0; m < NF; ++m)
#pragma unroll
            for (int it = 0; it < NV; ++it) {
                const int k = lane + 64 * it;
                v[m][it] = reinterpret_cast<const V4 *>(fl[m] + row0 * QD)[k < nvec ? k : 0];
            }
        T s = T(0);
#pragma unroll
        for (int m = 0; m < NF; ++m)
#pragma unroll
            for (int it = 0; it < NV; ++it) s += v[m][it][0];
        if constexpr (!(PARTS & 2)) {
            if (s == T(-12345)) Mo[lane] = s;          // keeps the loads (never true)
        }
        stage[lane] = s;
        __builtin_amdgcn_wave_barrier();
    } else if constexpr (PARTS & 1) {
        const int64_t N1 = g.N[1], N2 = g.pitch;          // grid lines of the fields may be padded
        const int64_t base = ((i1 * Q) * N1 + i2 * Q) * N2 + t0 * Q;
        const T *fl[NF] = {f0, f1, f2, f3};
        int64_t off[IT];
        bool ok[IT];
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int k = lane + 64 * it, gl = k / PER, e = (k - gl * PER) * U;
            ok[it] = k < TOT && e / Q < rows_here;
            off[it] = ok[it] ? base + (int64_t)(gl / Q) * N1 * N2 + (int64_t)(gl % Q) * N2 + e : base;
        }
        VT v[NF][IT];
#pragma unroll
        for (int m = 0; m < NF; ++m)
#pragma unroll
            for (int it = 0; it < IT; ++it) v[m][it] = *reinterpret_cast<const VT *>(fl[m] + off[it]);
        T s = T(0);
#pragma unroll
        for (int m = 0; m < NF; ++m)
#pragma unroll
            for (int it = 0; it < IT; ++it)
                if (ok[it]) s += v[m][it][0];
        if constexpr (!(PARTS & 2)) {
            if (s == T(-12345)) Mo[lane] = s;          // keeps the loads (never true)
        }
        stage[lane] = s;
        __builtin_amdgcn_wave_barrier();
    } else {
        for (int e = lane; e < OUT; e += 64) stage[e] = T(e);
        __builtin_amdgcn_wave_barrier();
    }
    if constexpr (PARTS & 2) {
        if ((flags & 3) == 3) {
            // each tile writes the whole 128-byte lines its output range touches (the lines
            // at its two ends also belong to the neighbouring tiles, which write them too):
            // the price of partial lines at tile boundaries; each store takes its value from
            // LDS, as in the kernel
            constexpr int LINE = 128 / (int)sizeof(T);
            constexpr int WRAP = R * SD >= 2048 ? 2048 : R * SD >= 1024 ? 1024 : 512;   // within stage
            const int64_t total = g.n[0] * g.n[1] * g.n[2] * (int64_t)SD;
            const int64_t lo = (row0 * SD) / LINE * LINE;
            int64_t hi = ((row0 + rows_here) * SD + LINE - 1) / LINE * LINE;
            hi = hi < total ? hi : total;
            const int nv = (int)((hi - lo) / VEC);
            for (int mat = 0; mat < 2; ++mat) {
                T *ob = (mat == 0 ? Mo : Ko) + lo;
                for (int k = lane; k < nv; k += 64)
                    __builtin_nontemporal_store(*reinterpret_cast<const VO *>(&stage[(k * VEC) & (WRAP - 1)]),
                                                reinterpret_cast<VO *>(ob + (int64_t)k * VEC));
                const int64_t t0v = lo + (int64_t)nv * VEC;
                if (lane < hi - t0v) (mat == 0 ? Mo : Ko)[t0v + lane] = T(0);
            }
            return;
        }
        const bool NT = sizeof(T) == 4 && !(flags & 1);
        const int nmat = (flags & 2) ? 1 : 2;
        const int n = rows_here * SD;
        const int shift = (int)((row0 * SD) & (VEC - 1));
        // the 16-byte stores start at the first 16-byte (or, flag 4, 128-byte) boundary of
        // the range; the values before it take one plain store per lane
        const int A = (flags & 4) ? 128 / (int)sizeof(T) : VEC;
        const int head = (int)((A - ((row0 * SD) & (A - 1))) & (A - 1));
        for (int mat = 0; mat < nmat; ++mat) {
            T *ob = (mat == 0 ? Mo : Ko) + row0 * SD;
            auto put = [](bool nt, auto v, auto *dst) {
                if (nt) __builtin_nontemporal_store(v, dst);
                else *dst = v;
            };
            if (lane < head && lane < n) put(NT, stage[shift + lane], ob + lane);
            const int nvec = (n - head) / VEC;
            for (int k = lane; k < nvec; k += 64) {
                const int e = head + k * VEC;
                const VO v = (flags & 8) ? VO{} : *reinterpret_cast<const VO *>(&stage[shift + e]);
                put(NT, v, reinterpret_cast<VO *>(ob + e));
            }
            const int tail0 = head + nvec * VEC;
            if (lane < n - tail0) put(NT, stage[shift + tail0 + lane], ob + tail0 + lane);
        }
    }
}

template <typename T, int P, int PARTS, int ORDER>
int launch_forward_probe(const Grid3 &g, const void *const *f, void *M, void *K, hipStream_t st, int flags) {
    constexpr int R = 64 / (2 * P + 1);
    const int tiles = (int)((g.n[2] + R - 1) / R);
    const int64_t tasks = g.n[0] * g.n[1] * tiles;
    if (tasks >= (int64_t(1) << 31) / 64) return -1;
    hipLaunchKernelGGL((forward_probe<T, P, PARTS, ORDER>), dim3((unsigned)tasks), dim3(64), 0, st, g, (const T *)f[0],
                       (const T *)f[1], (const T *)f[2], (const T *)f[3], (T *)M, (T *)K, tasks, tiles, flags);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

template <typename T, int P, int ORDER>
int forward_order(int parts, const Grid3 &g, const void *const *f, void *M, void *K, hipStream_t st, int flags) {
    switch (parts) {
        case 1: return launch_forward_probe<T, P, 1, ORDER>(g, f, M, K, st, flags);
        case 2: return launch_forward_probe<T, P, 2, ORDER>(g, f, M, K, st, flags);
        case 3: return launch_forward_probe<T, P, 3, ORDER>(g, f, M, K, st, flags);
        default: return -1;
    }
}

// parts: bits 0-1 as documented; bits 4-5 the work-group order (0: the kernel's runs of 8
// per XCD, 1: each XCD one contiguous share, 2: dispatch order, 3: runs of 128 per XCD)
template <typename T, int P>
int forward_parts(int parts, const Grid3 &g, const void *const *f, void *M, void *K, hipStream_t st) {
    // 1: ordinary stores, 2: M only, 3: whole lines; 4: 16-byte stores from line boundaries;
    // 8: 16-byte stores of constants
    const int flags = ((parts >> 6) & 3) | ((parts >> 8) & 12);
    switch ((parts >> 4) & 3) {
        case 0: return forward_order<T, P, 0>(parts & 3, g, f, M, K, st, flags);
        case 1: return forward_order<T, P, 1>(parts & 3, g, f, M, K, st, flags);
        case 2: return forward_order<T, P, 2>(parts & 3, g, f, M, K, st, flags);
        case 3: return forward_order<T, P, 3>(parts & 3, g, f, M, K, st, flags);
        default: return -1;
    }
}

bool geometry_ok(int dtype, int p, const int64_t *n_elem) {
    if ((dtype != 0 && dtype != 1) || (p != 2 && p != 3) || !n_elem) return false;
    for (int k = 0; k < 3; ++k)
        if (n_elem[k] < p + 1 || n_elem[k] > (int64_t(1) << 24)) return false;
    return true;
}

}  // namespace

extern "C" {

int wqap_stream(int what, void *dst, const void *src, int64_t n_bytes, void *stream) {
    if (what < 0 || what > 2 || n_bytes <= 0 || n_bytes % 16) return -1;
    if ((what != 1 && !dst) || (what != 0 && !src) || (what == 1 && !dst)) return -1;
    const int64_t n16 = n_bytes / 16;
    const int64_t blocks = std::min<int64_t>((n16 + 1023) / 1024, 256 * 64);   // grid-stride beyond
    hipLaunchKernelGGL(stream_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, what, (f4 *)dst,
                       (const f4 *)src, n16);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

int wqap_fronts(void *dst, int k, int64_t spacing, int64_t per_front, void *stream) {
    if (!dst || k < 1 || per_front < 4096 || per_front % 4096 || spacing % 16 || spacing < per_front) return -1;
    const int64_t blocks = std::min<int64_t>((per_front / 4096 * k + 3) / 4, 256 * 64);
    hipLaunchKernelGGL(fronts_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, (char *)dst, k, spacing,
                       per_front);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

int wqap_adjoint(int parts, int layout, int dtype, int p, const int64_t *n_elem, const void *gM, const void *gK,
                 void *const *out, void *stream) {
    if (!geometry_ok(dtype, p, n_elem) || layout < 0 || (layout & 63) > 49 || ((layout >> 6) & 3) > 2 ||
        layout >= 65536 || ((layout & (16384 | 32768)) && p != 3) || !out)
        return -1;
    if (((parts & 1) && (!gM || !gK)) || ((parts & 2) && (!out[0] || !out[1] || !out[2] || !out[3]))) return -1;
    const Grid3 g = grid_of(p, n_elem);
    hipStream_t st = (hipStream_t)stream;
    if (dtype == 0) return p == 2 ? adjoint_parts<float, 2>(parts, layout, g, gM, gK, out, st)
                                  : adjoint_parts<float, 3>(parts, layout, g, gM, gK, out, st);
    return p == 2 ? adjoint_parts<double, 2>(parts, layout, g, gM, gK, out, st)
                  : adjoint_parts<double, 3>(parts, layout, g, gM, gK, out, st);
}

int wqap_forward(int parts, int dtype, int p, const int64_t *n_elem, const void *const *fields, void *M, void *K,
                 void *stream) {
    if (!geometry_ok(dtype, p, n_elem) || !fields) return -1;
    if (((parts & 1) && (!fields[0] || !fields[1] || !fields[2] || !fields[3])) || ((parts & 2) && (!M || !K)) ||
        !M)
        return -1;
    Grid3 g = grid_of(p, n_elem);
    if (parts & 256) g.pitch = (g.N[2] + 31) / 32 * 32;      // fields with padded grid lines
    if (parts & 512) g.rowpts = 1;                           // fields stored row by row
    parts &= 255 | 1024 | 2048;
    hipStream_t st = (hipStream_t)stream;
    if (dtype == 0) return p == 2 ? forward_parts<float, 2>(parts, g, fields, M, K, st)
                                  : forward_parts<float, 3>(parts, g, fields, M, K, st);
    return p == 2 ? forward_parts<double, 2>(parts, g, fields, M, K, st)
                  : forward_parts<double, 3>(parts, g, fields, M, K, st);
}

}  // extern "C"
