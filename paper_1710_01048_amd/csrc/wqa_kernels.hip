// HIP kernels of libwqa for gfx950 (MI355X): row-wise weighted-quadrature assembly of
// the mass and stiffness matrices and its adjoint, sum-factorized one direction at a
// time (eq:Decompo) with each row's own rule tables (eq:GaussQuadSys,
// eq:GaussQuadSysStiff).
//
// Work decomposition (wave64, one wavefront = one tile of consecutive rows):
//   * A "line" fixes every row index but the last (i_1 for d = 2, (i_1, i_2) for d = 3);
//     a tile is R consecutive rows of one line, so the tables of the leading directions
//     are uniform across the wave and the coefficient samples of neighbouring rows are
//     neighbours in memory (row i owns grid points (i_k Q + q_k)_k, C order).
//   * Forward: lane (r, s_d) owns one slot column s_d of row r.  The tile's samples of
//     every field are staged in LDS with wide loads; each lane contracts its row's Q^d
//     samples over q_d against the table column s_d, then over q_{d-1}, ... in
//     registers, and finally over q_1 (the "final pass", selectable accumulation).  The
//     tile's whole output goes through LDS and leaves with 16-byte stores over one
//     contiguous range of the [row][S^d] output.
//   * Adjoint: lane (r, q_d) owns one node column of row r.  The upstream gradients
//     stream through a ring of s_1 slabs in LDS filled by direct global-to-LDS loads
//     (slots outside the space zeroed), are contracted over s_d, s_{d-1}, ..., and the
//     gradient of every sample is stored: on the grid directly (consecutive lanes =
//     consecutive grid points), stored row by row through LDS as whole blocks.
//   * Each kernel runs every line in one launch and picks the code path per wave: the
//     banded loops where the tile's leading indices are interior (leading tables banded),
//     the full loops elsewhere.
//   * Stiffness: term k uses the stiffness table in direction k and mass tables
//     elsewhere.  Forward terms with the mass table in direction 1 share the final
//     pass; adjoint terms with the mass table in direction d share the first pass.
#include "wqa_internal.h"

#include <algorithm>

namespace wqa {
namespace {

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// --- final-pass accumulators -------------------------------------------------------
// FINAL 0: plain fused multiply-add in T.
// FINAL 1: compensated dot product in FP32 registers (Ogita, Rump and Oishi's Dot2:
//          error-free products via FMA, error-free sums, errors summed separately).
// FINAL 2: mixed precision through an FP64 accumulator: the FP32 factor times the FP64
//          table entry, summed in FP64, rounded once (a v_fma_f64 issues at the FP32 rate).
template <typename T, int FINAL>
struct Acc {
    T s = T(0);
    __device__ __forceinline__ void add(T a, T b) { s = fma(a, b, s); }
    __device__ __forceinline__ T get() const { return s; }
};

template <>
struct Acc<float, 1> {
    float p = 0.f, e = 0.f;
    bool first = true;     // resolved at compile time in the unrolled loops
    // No contraction here: a multiply-add fused by the compiler (p + a * b as one FMA)
    // would break the error-free transformations, and could differ between call sites.
    __device__ __forceinline__ void add(float a, float b) {
#pragma clang fp contract(off)
        const float h = a * b;
        const float r = __builtin_fmaf(a, b, -h);      // a * b = h + r exactly
        if (first) {                                   // the sum so far is h itself
            p = h;
            e = r;
            first = false;
            return;
        }
        const float t = p + h;                         // p + h = t + q exactly
        const float z = t - p;
        const float q = (p - (t - z)) + (h - z);
        p = t;
        e += q + r;
    }
    __device__ __forceinline__ float get() const {
#pragma clang fp contract(off)
        return p + e;
    }
};

template <>
struct Acc<float, 2> {
    double s = 0.0;
    __device__ __forceinline__ void add(double a, float b) { s = __builtin_fma(a, (double)b, s); }
    __device__ __forceinline__ float get() const { return (float)s; }
};

// A copy of v the compiler cannot see through.  The adjoint's FP64-accumulated final pass
// passes each slab result through it at every use, so that the conversion to FP64 happens
// per use: one conversion shared by the outputs that read the same slab result would keep
// an FP64 copy of every live one (measured: 147 instead of 109 VGPRs in the banded kernel,
// 214 instead of 129 in the other).
template <typename T>
__device__ __forceinline__ T opaque(T v) {
    asm volatile("" : "+v"(v));
    return v;
}

// Table element type used by the final pass.
template <typename T, int FINAL> struct FinalTab { using type = T; };
template <> struct FinalTab<float, 2> { using type = double; };

// Table rows of the leading directions are the same for the whole wave; reading them
// through the constant address space lets them live in scalar registers even after the
// kernel has stored results (the tables are never written by a kernel).
template <typename T>
using cptr = const __attribute__((address_space(4))) T *;

template <typename T>
__device__ __forceinline__ cptr<T> table(const DevTabs &tb, int kind, int dir) {
    return (cptr<T>)(const T *)tb.t[kind][dir];
}

template <typename T, int FINAL>
__device__ __forceinline__ cptr<typename FinalTab<T, FINAL>::type> final_table(const DevTabs &tb, int kind, int dir) {
    if constexpr (FINAL == 2 && sizeof(T) == 4) return (cptr<double>)tb.t64[kind][dir];
    else return (cptr<T>)(const T *)tb.t[kind][dir];
}

__device__ __forceinline__ void phase_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
}

// Forces the values of a register array to be computed before this point (an empty asm
// that "modifies" them), so that later phases cannot delay the arithmetic that
// consumes the earlier phase's loads.
template <typename T, int A, int B>
__device__ __forceinline__ void pin(T (&V)[A][B]) {
#pragma unroll
    for (int a = 0; a < A; ++a)
#pragma unroll
        for (int b = 0; b < B; ++b) asm volatile("" : "+v"(V[a][b]));
}

template <typename T, int A, int B, int C>
__device__ __forceinline__ void pin(T (&V)[A][B][C]) {
#pragma unroll
    for (int a = 0; a < A; ++a) pin(V[a]);
}

template <typename T, int A>
__device__ __forceinline__ void pin(T (&V)[A]) {
#pragma unroll
    for (int a = 0; a < A; ++a) asm volatile("" : "+v"(V[a]));
}

template <typename T>
__device__ __forceinline__ void pin(T &v) {
    asm volatile("" : "+v"(v));
}

// Makes a wave-uniform table pointer opaque at this point: table reads through it are
// then issued after here instead of all being hoisted to the top of the kernel, which
// would keep every table value of every phase in scalar registers at once.
template <typename T>
__device__ __forceinline__ cptr<T> fresh(cptr<T> p) {
    asm volatile("" : "+s"(p));
    return p;
}

// Rows whose nodes sit one per element of their support, in order (every row but the p
// at each end of a direction, with the library's rules) have tables that vanish outside
// q <= s <= q + P: node q only meets the P+1 functions living on its element.  The
// banded code paths skip those zeros; the others run the full Q x S loops.  Both give
// bitwise the same sums.  The host checks the built tables and clears a direction's bit
// in DevSpace::band when a caller's rule breaks the pattern; tiles then take the full
// loops.
template <int P>
__device__ __forceinline__ constexpr bool in_band(int q, int s) {
    return s >= q && s <= q + P;
}

// Work-group index remapped so that each XCD takes one contiguous eighth of the grid: the
// hardware deals work-groups round-robin over the 8 XCDs (each with its own L2), and
// neighbouring tiles share the cache lines at their boundaries.
__device__ __forceinline__ uint32_t block_chunked() {
    const uint32_t b = blockIdx.x, nb = gridDim.x, q = nb / 8, r = nb % 8, x = b % 8, i = b / 8;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Work-group index remapped in runs of 8·G: within a run, XCD x takes the G consecutive
// indices x·G .. x·G+G-1, which it receives G dispatches apart.  Neighbouring tiles then
// share an L2 while the whole chip still sweeps one contiguous window of tiles (unlike
// block_chunked(), which gives each XCD its own eighth of the grid).  The incomplete
// last run keeps the identity, so the map is a permutation of [0, gridDim.x).
template <int G>
__device__ __forceinline__ uint32_t block_grouped() {
    const uint32_t b = blockIdx.x, span = 8u * G, full = gridDim.x / span * span;
    if (b >= full) return b;
    return b - b % span + (b % 8) * G + (b / 8) % G;
}

// Q consecutive staged samples from LDS.  Scalar reads on purpose: the lanes of one
// tile read R distinct rows at a time, which 16-byte reads serve with bank conflicts
// (measured slower than pairs of 4-byte reads).
template <typename T, int Q>
__device__ __forceinline__ void lds_q(const T *p, T (&v)[Q]) {
#pragma unroll
    for (int q = 0; q < Q; ++q) v[q] = p[q];
}

// Per-wave tile context shared by the forward and adjoint bodies.
struct Tile {
    int64_t i1, i2, t0, row0, il, nl;
    int rows_here, r;
    bool in_tile, active;
};

template <int D, int P>
__device__ __forceinline__ Tile make_tile(const DevSpace &sp, int64_t task, int tiles_per_line, int R,
                                          int lanes_per_row, int lane) {
    Tile t;
    // line (i_1 n_2) + i_2 (d = 3) or i_1 (d = 2), then the tile within it; 32-bit divisions
    // while the operands fit (64-bit ones take dozens of instructions)
    const int64_t line = task < INT32_MAX ? (int64_t)((uint32_t)task / (uint32_t)tiles_per_line) : task / tiles_per_line;
    const int tile = (int)(task - line * tiles_per_line);
    t.nl = sp.n[D - 1];
    if constexpr (D == 3) {
        t.i1 = (line < INT32_MAX && sp.n[1] < INT32_MAX) ? (int64_t)((uint32_t)line / (uint32_t)sp.n[1])
                                                          : line / sp.n[1];
        t.i2 = line - t.i1 * sp.n[1];
    } else {
        t.i1 = line;
        t.i2 = 0;
    }
    t.t0 = (int64_t)tile * R;
    t.rows_here = (int)((t.nl - t.t0) < R ? (t.nl - t.t0) : R);
    t.r = lane / lanes_per_row;
    t.in_tile = t.r < R;
    t.active = t.r < t.rows_here;
    t.il = t.t0 + (t.active ? t.r : 0);
    t.row0 = line * t.nl + t.t0;
    return t;
}

// Where the sample of point (q1[, q2], ql) of a lane's row lies in a sample buffer: a
// wave-uniform offset (uniform(q1, q2)) plus the lane's own (lo).  On the grid the row's
// point is ((i1 Q + q1), (i2 Q + q2), il Q + ql); stored row by row it is value
// ((q1 Q) + q2) Q + ql of the row's block of Q^d.
template <int D, int P>
struct SampleIndex {
    static constexpr int Q = P + 1, QD = (D == 3) ? Q * Q * Q : Q * Q;
    int64_t u0, s1, s2;    // uniform part: u0 + q1 s1 + q2 s2
    uint32_t lo;
    __device__ __forceinline__ SampleIndex(const DevSpace &sp, const Tile &t, int ql) {
        if (sp.rows) {
            u0 = t.row0 * QD;
            s1 = (D == 3) ? Q * Q : Q;
            s2 = Q;
            lo = (uint32_t)((t.il - t.t0) * QD + ql);
        } else {
            const int64_t N2 = (D == 3) ? sp.N[1] : sp.ld, N3 = (D == 3) ? sp.ld : 1;
            s1 = N2 * N3;
            s2 = N3;
            u0 = (D == 3) ? (t.i1 * Q * N2 + t.i2 * Q) * N3 : t.i1 * Q * N2;
            lo = (uint32_t)(t.il * Q + ql);
        }
    }
    __device__ __forceinline__ int64_t uniform(int q1, int q2) const { return u0 + q1 * s1 + q2 * s2; }
};

// Whether every leading index of the tile's line is interior and its direction's tables
// banded (see in_band).
template <int D, int P>
__device__ __forceinline__ bool tile_banded(const DevSpace &sp, const Tile &t) {
    bool b = (sp.band & 1) && t.i1 >= P && t.i1 < sp.n[0] - P;
    if constexpr (D == 3) b = b && (sp.band & 2) && t.i2 >= P && t.i2 < sp.n[1] - P;
    return b;
}

// --------------------------------------------------------------------------------------
// Forward.  Lane (r, s_d): row r of the tile, slot column s_d of the last direction.
template <typename T, int P, int D, int FINAL, bool BAND, int R>
struct Forward {
    static constexpr int Q = P + 1, S = 2 * P + 1;
    static constexpr int SL = (D == 3) ? S * S : S;
    static constexpr int SD = S * SL;
    using FT = typename FinalTab<T, FINAL>::type;

    const DevSpace &sp;
    const DevTabs &tb;
    const Tile &t;
    T *stage;          // this wave's staging buffer: the tile's samples, then its output
    int lane, sl;
    int64_t N2, N3;

    // Input staging: the samples of every field the tile needs go to LDS first, each
    // (q1[, q2]) line of the tile as one contiguous run of R rows x Q values, loaded with
    // a few wide, non-redundant loads that are all in flight at once (in registers, the
    // Q samples of a row would be loaded by each of its S lanes).
    static constexpr int NG = (D == 3) ? Q * Q : Q;     // lines per field
    static constexpr int FSZ = NG * R * Q;              // staged values per field

    template <int NF>
    __device__ __forceinline__ void stage_fields(const T *const (&f)[NF]) const {
        if (sp.rows) stage_rows<NF>(f);
        else stage_grid<NF>(f);
    }

    // Samples stored row by row: the tile's samples of a field are one contiguous block of
    // rows_here x Q^d values; value (r, g, q) of it (g the leading nodes, q the last one)
    // goes to the same LDS slot as from the grid, g R Q + r Q + q.
    template <int NF>
    __device__ __forceinline__ void stage_rows(const T *const (&f)[NF]) const {
        constexpr int QD = NG * Q;
        constexpr int U = (QD * (int)sizeof(T)) % 16 == 0 && Q % (16 / (int)sizeof(T)) == 0 ? 16 / (int)sizeof(T) : 1;
        constexpr int TOT = R * QD / U;                 // loads per field
        constexpr int IT = (TOT + 63) / 64;
        using VT = T __attribute__((ext_vector_type(U)));
        int lds[IT];
        bool ok[IT];
        const int n = t.rows_here * QD;
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int e = (lane + 64 * it) * U;
            const int r = e / QD, w = e - r * QD, g = w / Q;
            ok[it] = e < n;
            lds[it] = g * R * Q + r * Q + (w - g * Q);
        }
        const int64_t base = t.row0 * QD;
        VT v[NF][IT];
#pragma unroll
        for (int m = 0; m < NF; ++m)
#pragma unroll
            for (int it = 0; it < IT; ++it) {
                const int e = ok[it] ? (lane + 64 * it) * U : 0;
                v[m][it] = *reinterpret_cast<const VT *>(f[m] + base + e);
            }
#pragma unroll
        for (int m = 0; m < NF; ++m)
#pragma unroll
            for (int it = 0; it < IT; ++it)
                if (lane + 64 * it < TOT) *reinterpret_cast<VT *>(stage + m * FSZ + lds[it]) = ok[it] ? v[m][it] : VT(0);
    }

    template <int NF>
    __device__ __forceinline__ void stage_grid(const T *const (&f)[NF]) const {
        constexpr int U = (Q * (int)sizeof(T)) % 16 == 0 ? 16 / (int)sizeof(T) : 1;   // values per load
        constexpr int PER = R * Q / U;                  // loads per line
        constexpr int TOT = NG * PER;                   // loads per field
        constexpr int IT = (TOT + 63) / 64;
        using VT = T __attribute__((ext_vector_type(U)));
        int64_t off[IT];
        int lds[IT];
        bool ok[IT];
        const int64_t base = (D == 3) ? ((t.i1 * Q) * N2 + t.i2 * Q) * N3 + t.t0 * Q : (t.i1 * Q) * N2 + t.t0 * Q;
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int k = lane + 64 * it;
            const int g = k / PER, e = (k - g * PER) * U;   // line and first value in it
            ok[it] = k < TOT && e / Q < t.rows_here;
            int64_t loff;
            if constexpr (D == 3) loff = (int64_t)(g / Q) * N2 * N3 + (int64_t)(g % Q) * N3;
            else loff = (int64_t)g * N2;
            off[it] = ok[it] ? base + loff + e : base;
            lds[it] = g * R * Q + e;
        }
        VT v[NF][IT];
#pragma unroll
        for (int m = 0; m < NF; ++m)
#pragma unroll
            for (int it = 0; it < IT; ++it) v[m][it] = *reinterpret_cast<const VT *>(f[m] + off[it]);
#pragma unroll
        for (int m = 0; m < NF; ++m)
#pragma unroll
            for (int it = 0; it < IT; ++it)
                if (lane + 64 * it < TOT) *reinterpret_cast<VT *>(stage + m * FSZ + lds[it]) = ok[it] ? v[m][it] : VT(0);
    }

    // V[s2][q1] = sum_{q2} sum_{q3} f[q1][q2][q3] t3[q3][sl] t2[q2][s2]     (d = 3)
    // V[0][q1]  = sum_{q2} f[q1][q2] t2[q2][sl]                            (d = 2)
    // Samples come from the staged field slot fi.
    __device__ __forceinline__ void contract(int fi, const T *t_last, cptr<T> t2, T (&V)[S][Q],
                                             bool accumulate) const {
        T tl[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) tl[q] = t_last[q * S + sl];
        const T *fs = stage + fi * FSZ + (t.r < t.rows_here ? t.r : 0) * Q;
        t2 = fresh(t2);
        if constexpr (D == 3) {
#pragma unroll
            for (int q1 = 0; q1 < Q; ++q1) {
                T U[Q];
#pragma unroll
                for (int q2 = 0; q2 < Q; ++q2) {
                    T v[Q];
                    lds_q<T, Q>(fs + (q1 * Q + q2) * R * Q, v);
                    T acc = T(0);
#pragma unroll
                    for (int q3 = 0; q3 < Q; ++q3) acc = fma(v[q3], tl[q3], acc);
                    U[q2] = acc;
                }
#pragma unroll
                for (int s2 = 0; s2 < S; ++s2) {
                    T acc = accumulate ? V[s2][q1] : T(0);
#pragma unroll
                    for (int q2 = 0; q2 < Q; ++q2)
                        if (!BAND || in_band<P>(q2, s2)) acc = fma(U[q2], t2[q2 * S + s2], acc);
                    V[s2][q1] = acc;
                }
            }
        } else {
#pragma unroll
            for (int q1 = 0; q1 < Q; ++q1) {
                T v[Q];
                lds_q<T, Q>(fs + q1 * R * Q, v);
                T acc = accumulate ? V[0][q1] : T(0);
#pragma unroll
                for (int q2 = 0; q2 < Q; ++q2) acc = fma(v[q2], tl[q2], acc);
                V[0][q1] = acc;
            }
        }
    }

    // Final pass over q1 and store: X[s1][s2][sl] = sum_q1 fa[q1][s1] Va[s2][q1]
    // (+ fb[q1][s1] Vb[s2][q1]).  Slots whose column leaves the space come out as exact
    // zeros without a test: the table factor of that column is 0 in its direction.  The
    // whole tile (rows_here x S^d values, one contiguous range of the output) goes to LDS,
    // shifted so that LDS and global addresses share their alignment, then leaves with
    // 16-byte stores.
    template <bool TWO>
    __device__ __forceinline__ void emit(cptr<FT> fa, const T (&Va)[S][Q], cptr<FT> fb, const T (&Vb)[S][Q],
                                         T *__restrict__ out) const {
        constexpr int NS2 = (D == 3) ? S : 1;
        constexpr int VEC = 16 / (int)sizeof(T);
        const int shift = (int)((t.row0 * SD) & (VEC - 1));
#pragma unroll
        for (int s1 = 0; s1 < S; ++s1) {
            fa = fresh(fa);
            if constexpr (TWO) fb = fresh(fb);
            if (t.in_tile) {
#pragma unroll
                for (int s2 = 0; s2 < NS2; ++s2) {
                    Acc<T, FINAL> acc;
#pragma unroll
                    for (int q1 = 0; q1 < Q; ++q1) {
                        if (!BAND || in_band<P>(q1, s1)) {
                            acc.add(fa[q1 * S + s1], Va[s2][q1]);
                            if constexpr (TWO) acc.add(fb[q1 * S + s1], Vb[s2][q1]);
                        }
                    }
                    stage[shift + t.r * SD + s1 * SL + s2 * S + sl] = acc.get();
                }
            }
        }
        // FP32 streams the output past the caches with nontemporal stores (it is not read
        // again here; measured 2-7% faster); FP64 measured faster with ordinary stores.
        constexpr bool NT = sizeof(T) == 4;
        using V = T __attribute__((ext_vector_type(VEC)));
        auto put = [](auto v, auto *dst) {
            if constexpr (NT) __builtin_nontemporal_store(v, dst);
            else *dst = v;
        };
        wave_lds_sync();
        const int n = t.rows_here * SD;
        T *ob = out + t.row0 * SD;
        const int head = (VEC - shift) & (VEC - 1);
        if (lane < head && lane < n) put(stage[shift + lane], ob + lane);
        const int nvec = (n - head) / VEC;
        for (int k = lane; k < nvec; k += 64) {
            const int e = head + k * VEC;
            put(*reinterpret_cast<const V *>(&stage[shift + e]), reinterpret_cast<V *>(ob + (uint32_t)e));
        }
        const int tail0 = head + nvec * VEC;
        if (lane < n - tail0) put(stage[shift + tail0 + lane], ob + (uint32_t)(tail0 + lane));
        wave_lds_sync();
    }
};

template <typename T, int P, int D, int WHAT, int FINAL, bool BAND, int R>
__device__ __forceinline__ void forward_body(const DevSpace &sp, const DevTabs &tb, const Tile &t, T *stage,
                                             int lane, const T *__restrict__ cf, const T *__restrict__ a0,
                                             const T *__restrict__ a1, const T *__restrict__ a2,
                                             T *__restrict__ Mo, T *__restrict__ Ko) {
    using F = Forward<T, P, D, FINAL, BAND, R>;
    constexpr int Q = F::Q, S = F::S;
    using FT = typename F::FT;
    F fw{sp, tb, t, stage, lane, lane - t.r * S, (D == 3) ? sp.N[1] : sp.ld, (D == 3) ? sp.ld : 1};
    const int64_t rs = (int64_t)Q * S;
    cptr<T> M2 = table<T>(tb, 0, 1) + (D == 3 ? t.i2 : 0) * rs;
    cptr<T> K2 = table<T>(tb, 1, 1) + (D == 3 ? t.i2 : 0) * rs;
    const T *ML = (const T *)tb.t[0][D - 1] + t.il * rs;
    const T *KL = (const T *)tb.t[1][D - 1] + t.il * rs;
    cptr<FT> fM1 = final_table<T, FINAL>(tb, 0, 0) + t.i1 * rs;
    cptr<FT> fK1 = final_table<T, FINAL>(tb, 1, 0) + t.i1 * rs;
    // Every field is contracted before the first output is written (the outputs reuse the
    // staging buffer).  The pins and phase barriers keep the phases in order: the empty
    // asm with a memory clobber stops loads from being hoisted across it, the scheduling
    // barrier stops the machine scheduler from interleaving.
    constexpr bool DO_M = (WHAT & kWhatM) != 0, DO_K = (WHAT & kWhatK) != 0;
    constexpr int NF = (DO_M ? 1 : 0) + (DO_K ? D : 0);
    const int fk = DO_M ? 1 : 0;                  // field slot of a_1
    {
        const T *fl[NF];
        if constexpr (DO_M) fl[0] = cf;
        if constexpr (DO_K) {
            fl[fk] = a0;
            fl[fk + 1] = a1;
            if constexpr (D == 3) fl[fk + 2] = a2;
        }
        fw.template stage_fields<NF>(fl);
        wave_lds_sync();
    }
    T V[DO_M ? S : 1][Q], V1[DO_K ? S : 1][Q], V2[DO_K ? S : 1][Q];
    if constexpr (DO_M) {
        fw.contract(0, ML, M2, V, false);
        pin(V);
        phase_barrier();
    }
    if constexpr (DO_K) {
        if constexpr (D == 3) {
            fw.contract(fk, ML, M2, V1, false);           // term 1: stiffness table in direction 1
            pin(V1);
            phase_barrier();
            fw.contract(fk + 1, ML, K2, V2, false);       // term 2: stiffness table in direction 2
            pin(V2);
            phase_barrier();
            fw.contract(fk + 2, KL, M2, V2, true);        // term 3: stiffness table in direction 3
        } else {
            fw.contract(fk, ML, M2, V1, false);           // term 1: stiffness table in direction 1
            pin(V1);
            phase_barrier();
            fw.contract(fk + 1, KL, M2, V2, false);       // term 2: stiffness table in direction 2
        }
        pin(V2);
        phase_barrier();
    }
    wave_lds_sync();                                      // every lane done reading the samples
    if constexpr (DO_M) {
        fw.template emit<false>(fM1, V, fM1, V, Mo);
        phase_barrier();
    }
    if constexpr (DO_K) {
        fw.template emit<true>(fK1, V1, fM1, V2, Ko);
    }
}

template <typename T, int P, int D, int WHAT, int FINAL, int WPB, int R>
__global__ __launch_bounds__(64 * WPB) void forward_kernel(
    DevSpace sp, DevTabs tb, const T *__restrict__ cf, const T *__restrict__ a0,
    const T *__restrict__ a1, const T *__restrict__ a2, T *__restrict__ Mo,
    T *__restrict__ Ko, int64_t task0, int64_t n_tasks, int tiles_per_line) {
    constexpr int S = 2 * P + 1;                   // R: rows per wave tile (<= 64 / S)
    constexpr int SL = (D == 3) ? S * S : S;
    constexpr int Q = P + 1, NG = (D == 3) ? Q * Q : Q;
    constexpr int NF = ((WHAT & kWhatM) ? 1 : 0) + ((WHAT & kWhatK) ? D : 0);
    constexpr int OUT = R * S * SL + 16 / (int)sizeof(T), IN = NF * NG * R * Q;
    __shared__ __align__(16) T stage[WPB][OUT > IN ? OUT : IN];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));   // uniform per wave
    const int lane = (int)(threadIdx.x & 63);
    // runs of 8 tiles per XCD on the grid (neighbouring tiles share the cache lines of
    // their sample runs); samples stored row by row share none, and runs of 128 tiles per
    // XCD measured 2-3% faster there (160^3 and 96^3)
    const int64_t task = task0 + (int64_t)(sp.rows ? block_grouped<128>() : block_grouped<8>()) * WPB + wave;
    if (task >= n_tasks) return;                   // whole wave leaves; no block barriers below
    const Tile t = make_tile<D, P>(sp, task, tiles_per_line, R, S, lane);
    if (tile_banded<D, P>(sp, t))
        forward_body<T, P, D, WHAT, FINAL, true, R>(sp, tb, t, stage[wave], lane, cf, a0, a1, a2, Mo, Ko);
    else
        forward_body<T, P, D, WHAT, FINAL, false, R>(sp, tb, t, stage[wave], lane, cf, a0, a1, a2, Mo, Ko);
}

// --------------------------------------------------------------------------------------
// Adjoint.  Lane (r, q_d): row r of the tile, node column q_d of the last direction.
// The upstream gradients of the tile stream through a ring of RING slab buffers in this
// wave's LDS: one buffer holds one s1 slab (R rows x S^(d-1) values), filled by direct
// global-to-LDS loads, so no registers hold the data in flight.  Slab pos + RING - 1 is
// issued when slab pos is taken up, then the wave waits for slab pos alone; the later
// slabs stay in flight while it is contracted (see acquire()).  The stream is gM's slabs,
// then gK's.  Each slab reduces to Z[s1][q2] in registers; the final pass over s1 gives
// every output, stored directly on the grid or through LDS as row blocks.
typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void glb_void_t;

// Waits until at most N vector-memory operations of this wave are in flight.  They
// complete in issue order, so this waits for everything issued before the last N.
template <int N>
__device__ __forceinline__ void wait_vm() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// S consecutive values of a ring slab (LDS byte address a, aligned to the value size),
// read in one asm block that also waits for them.  The compiler treats any LDS read as
// possibly aliasing a pending direct-to-LDS load and puts its own vmcnt(0) wait before it;
// acquire() waits for the slab it hands out, and these reads keep the compiler from
// adding a wait for the slabs still in flight.
template <typename T, int S>
__device__ __forceinline__ void lds_row(uint32_t a, T (&g)[S]) {
    static_assert(S == 5 || S == 7, "rows of 2p+1 values, p = 2 or 3");
    using T2 = T __attribute__((ext_vector_type(2)));
    T2 x0, x1, x2;
    T x3;
    if constexpr (sizeof(T) == 4 && S == 7) {
        asm volatile(
            "ds_read2_b32 %0, %4 offset1:1\n\t"
            "ds_read2_b32 %1, %4 offset0:2 offset1:3\n\t"
            "ds_read2_b32 %2, %4 offset0:4 offset1:5\n\t"
            "ds_read_b32 %3, %4 offset:24\n\t"
            "s_waitcnt lgkmcnt(0)"
            : "=&v"(x0), "=&v"(x1), "=&v"(x2), "=&v"(x3) : "v"(a) : "memory");
    } else if constexpr (sizeof(T) == 4) {
        asm volatile(
            "ds_read2_b32 %0, %3 offset1:1\n\t"
            "ds_read2_b32 %1, %3 offset0:2 offset1:3\n\t"
            "ds_read_b32 %2, %3 offset:16\n\t"
            "s_waitcnt lgkmcnt(0)"
            : "=&v"(x0), "=&v"(x1), "=&v"(x3) : "v"(a) : "memory");
    } else if constexpr (S == 7) {
        asm volatile(
            "ds_read2_b64 %0, %4 offset1:1\n\t"
            "ds_read2_b64 %1, %4 offset0:2 offset1:3\n\t"
            "ds_read2_b64 %2, %4 offset0:4 offset1:5\n\t"
            "ds_read_b64 %3, %4 offset:48\n\t"
            "s_waitcnt lgkmcnt(0)"
            : "=&v"(x0), "=&v"(x1), "=&v"(x2), "=&v"(x3) : "v"(a) : "memory");
    } else {
        asm volatile(
            "ds_read2_b64 %0, %3 offset1:1\n\t"
            "ds_read2_b64 %1, %3 offset0:2 offset1:3\n\t"
            "ds_read_b64 %2, %3 offset:32\n\t"
            "s_waitcnt lgkmcnt(0)"
            : "=&v"(x0), "=&v"(x1), "=&v"(x3) : "v"(a) : "memory");
    }
    g[0] = x0.x;
    g[1] = x0.y;
    g[2] = x1.x;
    g[3] = x1.y;
    if constexpr (S == 7) {
        g[4] = x2.x;
        g[5] = x2.y;
    }
    g[S - 1] = x3;
}

// P+1 consecutive values of a ring slab at a per-lane address, read and waited for like
// lds_row: the band s = q .. q+P of one slab row that a lane with node q meets when the
// row's last-direction table is banded.
template <typename T, int P>
__device__ __forceinline__ void lds_band(uint32_t a, T (&g)[P + 1]) {
    static_assert(P == 2 || P == 3, "p = 2 or 3");
    using T2 = T __attribute__((ext_vector_type(2)));
    T2 x0, x1;
    T x2;
    if constexpr (sizeof(T) == 4 && P == 3) {
        asm volatile(
            "ds_read2_b32 %0, %2 offset1:1\n\t"
            "ds_read2_b32 %1, %2 offset0:2 offset1:3\n\t"
            "s_waitcnt lgkmcnt(0)"
            : "=&v"(x0), "=&v"(x1) : "v"(a) : "memory");
        g[2] = x1.x;
        g[3] = x1.y;
    } else if constexpr (sizeof(T) == 4) {
        asm volatile(
            "ds_read2_b32 %0, %2 offset1:1\n\t"
            "ds_read_b32 %1, %2 offset:8\n\t"
            "s_waitcnt lgkmcnt(0)"
            : "=&v"(x0), "=&v"(x2) : "v"(a) : "memory");
        g[2] = x2;
    } else if constexpr (P == 3) {
        asm volatile(
            "ds_read2_b64 %0, %2 offset1:1\n\t"
            "ds_read2_b64 %1, %2 offset0:2 offset1:3\n\t"
            "s_waitcnt lgkmcnt(0)"
            : "=&v"(x0), "=&v"(x1) : "v"(a) : "memory");
        g[2] = x1.x;
        g[3] = x1.y;
    } else {
        asm volatile(
            "ds_read2_b64 %0, %2 offset1:1\n\t"
            "ds_read_b64 %1, %2 offset:16\n\t"
            "s_waitcnt lgkmcnt(0)"
            : "=&v"(x0), "=&v"(x2) : "v"(a) : "memory");
        g[2] = x2;
    }
    g[0] = x0.x;
    g[1] = x0.y;
}

template <typename T>
__device__ __forceinline__ uint32_t lds_addr(const T *p) {
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) T *)p;
}

// LB: every row of the tile is at least P from both ends of its line and the last
// direction's tables are banded, so a lane with node q_d only meets the slots
// s_d = q_d .. q_d + P of each slab row (tl then holds those P+1 table entries).
template <typename T, int P, int D, int FINAL, bool BAND, int WPB, int R, int RING, bool LB = false,
          bool ROWS = false>
struct Adjoint {
    static constexpr int Q = P + 1, S = 2 * P + 1;
    static constexpr int SL = (D == 3) ? S * S : S;     // slots of one s1 slab
    static constexpr int SD = S * SL;
    static constexpr int U = (int)sizeof(T) / 4;        // dwords per value
    static constexpr int NE = R * SL * U;               // dwords of one slab
    static constexpr int NPF = (NE + 63) / 64;          // loads per lane per slab
    static constexpr int SLOT = 64 * NPF;               // dwords per ring buffer
    static constexpr int NQ2 = (D == 3) ? Q : 1;
    using FT = typename FinalTab<T, FINAL>::type;
    static_assert(NPF <= 32, "one validity bit per load");
    static_assert(RING >= 2 && RING <= 4 && (RING - 1) * NPF < 64, "ring depth");
    static constexpr bool LIMIT = sizeof(T) == 8;
    static constexpr int NT = LB ? P + 1 : S;            // last-direction table entries per lane
    // Samples stored row by row: the tile's gradients leave through LDS staging in the
    // ring -- before the stream's last slab through the buffer of the run's last slab (free
    // from its contraction until the next matrix's first acquire refills it), CH rows of
    // one field at a time; after it through the whole ring.
    static constexpr int QD = (D == 3) ? Q * Q * Q : Q * Q;
    static constexpr int CH = (SLOT * 4 / (int)sizeof(T)) / QD < R ? (SLOT * 4 / (int)sizeof(T)) / QD : R;
    static_assert(CH >= 1, "a ring buffer holds at least one row of gradients");

    const DevSpace &sp;
    const Tile &t;
    uint32_t *ring;    // RING * SLOT dwords of this wave
    int lane, ql;
    const T *gM, *gK;
    int s1_lo, n_s1, nM, n_tot;   // slabs per matrix, gM's slabs in the stream, all slabs
    bool fix;                     // the tile has slots outside the space (zeroed after loading)

    // Per-lane gather map of one slab, the same for every s1 and both matrices: dword k of
    // this lane (d = lane + 64 k) is half d % U of value e = d / U, slot tt of tile row rr
    // (e = rr * SL + tt); goff is its dword offset from the slab's first value.  Values
    // outside the space or beyond the tile's rows load the slab's first value instead (an
    // address that always exists) and have their validity bit clear.
    uint32_t goff[NPF];
    uint32_t valid;

    __device__ __forceinline__ void make_map() {
        valid = 0;
        const int i2 = (int)t.i2, t0 = (int)t.t0, nl = (int)t.nl, n2 = (int)sp.n[1];
#pragma unroll
        for (int k = 0; k < NPF; ++k) {
            const int dw = lane + 64 * k;
            const int e = dw / U, half = dw - e * U;
            const int rr = e / SL, tt = e - rr * SL;
            const int s2 = (D == 3) ? tt / S : 0, s3 = (D == 3) ? tt - (tt / S) * S : tt;
            bool ok = dw < NE && rr < t.rows_here;
            if constexpr (D == 3) {
                const int j2 = i2 - P + s2, j3 = t0 + rr - P + s3;
                ok = ok && j2 >= 0 && j2 < n2 && j3 >= 0 && j3 < nl;
            } else {
                const int j2 = t0 + rr - P + s3;
                ok = ok && j2 >= 0 && j2 < nl;
            }
            goff[k] = ok ? (uint32_t)((rr * SD + tt) * U + half) : 0u;
            valid |= (ok ? 1u : 0u) << k;
        }
        pin(goff);
        asm volatile("" : "+v"(valid));
    }

    __device__ __forceinline__ void issue(int pos) const {
        const bool first = pos < nM;
        const T *g = first ? gM : gK;
        const int s1 = s1_lo + (first ? pos : pos - nM);
        const uint32_t *src = reinterpret_cast<const uint32_t *>(g + (t.row0 * SD + (int64_t)s1 * SL));
        uint32_t *dst = ring + (pos % RING) * SLOT;
#pragma unroll
        for (int k = 0; k < NPF; ++k)
            __builtin_amdgcn_global_load_lds((glb_void_t *)(src + goff[k]), (lds_void_t *)(dst + 64 * k), 4, 0, 0);
    }

    // Waits for the slab issued `after` slabs before the newest one.
    __device__ __forceinline__ void wait_slab(int after) const {
        if constexpr (RING >= 4) {
            if (after >= 3) { wait_vm<3 * NPF>(); return; }
        }
        if constexpr (RING >= 3) {
            if (after >= 2) { wait_vm<2 * NPF>(); return; }
        }
        if (after >= 1) { wait_vm<NPF>(); return; }
        wait_vm<0>();
    }

    // Makes slab `pos` of the stream readable: refills the buffer read last (its reads are
    // complete) with slab pos + RING - 1, waits for slab pos (vector memory operations
    // complete in issue order, so a count of outstanding loads names the slabs still in
    // flight) and zeroes its slots outside the space; the later slabs stay in flight while
    // this one is contracted.  (Waiting for every load instead measured 6% slower in FP32
    // at 160^3 and 10% at 96^3, the same in FP64.)  Every lane takes part.
    __device__ __forceinline__ const T *acquire(int pos) const {
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        if (pos + RING - 1 < n_tot) issue(pos + RING - 1);
        const int left = n_tot - 1 - pos;
        wait_slab(left < RING - 1 ? left : RING - 1);
        uint32_t *slot = ring + (pos % RING) * SLOT;
        if (fix) {
#pragma unroll
            for (int k = 0; k < NPF; ++k)
                if (!((valid >> k) & 1u) && (64 * (k + 1) <= NE || lane + 64 * k < NE)) slot[64 * k + lane] = 0u;
        }
        wave_lds_sync();
        return reinterpret_cast<const T *>(slot);
    }

    // Z[zi][q2] (+)= sum_{s2} (sum_{s3} G[s1][s2][s3] tl[s3]) t2[q2][s2] for NSET sets that
    // share the slab (tl[m], t2[m]); d = 2: Z[zi][0] = sum_{s2} G[s1][s2] tl[s2].
    template <int NSET, int NZ>
    __device__ __forceinline__ void slab_contract(const T *slab, int zi, const T (&tl)[NSET][NT],
                                                  const cptr<T> (&t2)[NSET], T (&Z)[NSET][NZ][NQ2]) const {
        const T *row = slab + (t.r < t.rows_here ? t.r : 0) * SL + (LB ? ql : 0);
        if constexpr (D == 3) {
#pragma unroll
            for (int s2 = 0; s2 < S; ++s2) {
                T g[NT];
                if constexpr (LB) lds_band<T, P>(lds_addr(row + s2 * S), g);
                else lds_row<T, S>(lds_addr(row + s2 * S), g);
                // the table entries of one s2 at a time in scalar registers (a whole slab's
                // would not fit beside everything else)
                cptr<T> t2r[NSET];
#pragma unroll
                for (int m = 0; m < NSET; ++m) t2r[m] = fresh(t2[m]);
#pragma unroll
                for (int m = 0; m < NSET; ++m) {
                    T y = T(0);
#pragma unroll
                    for (int s3 = 0; s3 < NT; ++s3) y = fma(g[s3], tl[m][s3], y);
#pragma unroll
                    for (int q2 = 0; q2 < Q; ++q2)
                        if (!BAND || in_band<P>(q2, s2)) Z[m][zi][q2] = fma(y, t2r[m][q2 * S + s2], Z[m][zi][q2]);
                }
                // one s2 row of the slab at a time: the scheduler would otherwise hold the
                // whole row of the slab in registers
                if constexpr (LIMIT) __builtin_amdgcn_sched_barrier(0);
            }
        } else {
            T g[NT];
            if constexpr (LB) lds_band<T, P>(lds_addr(row), g);
            else lds_row<T, S>(lds_addr(row), g);
#pragma unroll
            for (int m = 0; m < NSET; ++m) {
                T y = T(0);
#pragma unroll
                for (int s2 = 0; s2 < NT; ++s2) y = fma(g[s2], tl[m][s2], y);
                Z[m][zi][0] = y;
            }
        }
    }

    // Final pass of one q1 (compensated or FP64-accumulated, s1 ascending) and its stores.
    template <int NSET, int NZ>
    __device__ __forceinline__ void emit_q1(int q1, const cptr<FT> (&f1)[NSET], const T (&Z)[NSET][NZ][NQ2],
                                            T *const (&out)[NSET]) const {
        const int64_t N2 = (D == 3) ? sp.N[1] : sp.ld, N3 = (D == 3) ? sp.ld : 1;
        const uint32_t lo = (uint32_t)(t.il * Q + ql);
#pragma unroll
        for (int m = 0; m < NSET; ++m) {
            const cptr<FT> f1m = fresh(f1[m]);
#pragma unroll
            for (int q2 = 0; q2 < NQ2; ++q2) {
                Acc<T, FINAL> a;
#pragma unroll
                for (int s1 = 0; s1 < S; ++s1)
                    if (!BAND || in_band<P>(q1, s1)) a.add(f1m[q1 * S + s1], fin(Z[m][s1][q2]));
                int64_t off;     // wave-uniform part; the lane adds il * Q + ql
                if constexpr (D == 3) off = ((t.i1 * Q + q1) * N2 + t.i2 * Q + q2) * N3;
                else off = (t.i1 * Q + q1) * N2;
                (out[m] + off)[lo] = a.get();
            }
        }
    }

    // a slab result as the final pass takes it (see opaque)
    static __device__ __forceinline__ T fin(T z) {
        if constexpr (FINAL == 2 && sizeof(T) == 4) return opaque(z);
        else return z;
    }

    // Samples stored row by row: the values val(m, q1, q2) of each lane's point column go
    // to a staging buffer in LDS -- value w = (q1 Q + q2) Q + ql of row r at
    // r QD + (w ^ swz(r)), a swizzle that spreads one store instruction over the banks --
    // and the tile's block of rows_here x QD values of each field leaves with 16-byte
    // stores, consecutive lanes at consecutive addresses.
    static __device__ __forceinline__ int swz(int r) {
        constexpr int MASK = (QD & (QD - 1)) == 0 && QD >= 16 ? (QD / 4 < 16 ? QD / 4 : 16) - 1 : 0;
        return (r & MASK) << 2;
    }

    // NF fields and CHX rows per round: the lanes of those rows put their values in buf,
    // then the wave stores each field's CHX rows as one contiguous block.
    template <int NSET, int NF, int CHX, class F>
    __device__ __forceinline__ void stage_out(T *buf, F val, T *const (&out)[NSET]) const {
        constexpr int VEC = (QD * (int)sizeof(T)) % 16 == 0 ? 16 / (int)sizeof(T) : 1;
        using V = T __attribute__((ext_vector_type(VEC)));
#pragma unroll
        for (int m0 = 0; m0 < NSET; m0 += NF) {
#pragma unroll
            for (int c0 = 0; c0 < R; c0 += CHX) {
                const int rr = t.r - c0;
                if (t.active && rr >= 0 && rr < CHX) {
#pragma unroll
                    for (int mm = 0; mm < NF && m0 + mm < NSET; ++mm)
#pragma unroll
                        for (int q1 = 0; q1 < Q; ++q1)
#pragma unroll
                            for (int q2 = 0; q2 < NQ2; ++q2)
                                buf[(mm * CHX + rr) * QD + (((q1 * NQ2 + q2) * Q + ql) ^ swz(rr))] = val(m0 + mm, q1, q2);
                }
                wave_lds_sync();
                const int nr = t.rows_here - c0 < CHX ? t.rows_here - c0 : CHX;
                if (nr > 0) {
                    const int nv = nr * QD / VEC;
#pragma unroll
                    for (int mm = 0; mm < NF && m0 + mm < NSET; ++mm) {
                        T *dst = out[m0 + mm] + (t.row0 + c0) * QD;
                        const T *src = buf + mm * CHX * QD;
                        for (int k = lane; k < nv; k += 64) {
                            const int e = k * VEC, r = e / QD, w = e - r * QD;
                            *reinterpret_cast<V *>(dst + e) = *reinterpret_cast<const V *>(src + r * QD + (w ^ swz(r)));
                        }
                    }
                }
                wave_lds_sync();
            }
        }
    }

    // The run's gradients, val(m, q1, q2) for the lane's point column.  Before the stream's
    // last slab only the ring buffer of the run's last slab is free (one field and CH rows
    // per round); after it the whole ring is, and every field goes through it together,
    // CHA rows per round (FP32 cubic: the whole tile in one round).
    template <int NSET, class F>
    __device__ __forceinline__ void store_rows(int pos_last, F val, T *const (&out)[NSET]) const {
        constexpr int CAP = RING * SLOT * 4 / (int)sizeof(T) / (NSET * QD);
        constexpr int CHA = CAP < R ? CAP : R;
        if constexpr (CHA >= 1) {
            if (pos_last == n_tot - 1) {
                stage_out<NSET, NSET, CHA>(reinterpret_cast<T *>(ring), val, out);
                return;
            }
        }
        stage_out<NSET, 1, CH>(reinterpret_cast<T *>(ring + (pos_last % RING) * SLOT), val, out);
    }

    // Final pass of output (m, q1, q2): sum over s1 of the first-direction table entry times
    // the slab result, s1 ascending.
    template <int NSET, int NZ>
    __device__ __forceinline__ T final_q1(const cptr<FT> &f1m, int q1, int q2, const T (&Z)[NSET][NZ][NQ2],
                                          int m) const {
        Acc<T, FINAL> a;
#pragma unroll
        for (int s1 = 0; s1 < S; ++s1)
            if (!BAND || in_band<P>(q1, s1)) a.add(f1m[q1 * S + s1], fin(Z[m][s1][q2]));
        return a.get();
    }

    // The slabs of one matrix (stream positions pos0 ...), then the final pass over s1 and
    // the stores.  Plain accumulation (FINAL 0, and every FP64 call) keeps running sums
    // over s1, Q x Q per set; the FP32 compensated and FP64-accumulated passes keep the
    // S x Q slab results Z[s1][q2] and sum them at the end.
    template <int NSET>
    __device__ __forceinline__ void run(int pos0, const T (&tl)[NSET][NT], const cptr<T> (&t2)[NSET],
                                        const cptr<FT> (&f1)[NSET], T *const (&out)[NSET]) const {
        constexpr bool RUNNING = (FINAL == 0);
        constexpr int NZ = RUNNING ? 1 : S;
        constexpr bool EARLY = BAND && !RUNNING;         // outputs final once s1 = q1 + P
        T Z[NSET][NZ][NQ2];
        T acc[NSET][RUNNING ? Q : 1][NQ2];
        T O[NSET][EARLY && ROWS ? Q : 1][NQ2];          // finished outputs held for the block store
#pragma unroll
        for (int m = 0; m < NSET; ++m) {
#pragma unroll
            for (int z = 0; z < NZ; ++z)
#pragma unroll
                for (int q2 = 0; q2 < NQ2; ++q2) Z[m][z][q2] = T(0);
#pragma unroll
            for (int z = 0; z < (RUNNING ? Q : 1); ++z)
#pragma unroll
                for (int q2 = 0; q2 < NQ2; ++q2) acc[m][z][q2] = T(0);
        }
        const int s1_hi = s1_lo + n_s1 - 1;
#pragma unroll
        for (int s1 = 0; s1 < S; ++s1) {
            if (s1 < s1_lo || s1 > s1_hi) continue;     // slab outside the space: contributes 0
            const T *slab = acquire(pos0 + s1 - s1_lo);
            cptr<T> t2s[NSET];
            cptr<FT> f1s[NSET];
#pragma unroll
            for (int m = 0; m < NSET; ++m) {
                t2s[m] = fresh(t2[m]);
                f1s[m] = fresh(f1[m]);
            }
            if (t.in_tile) {
                if constexpr (RUNNING) {
#pragma unroll
                    for (int m = 0; m < NSET; ++m)
#pragma unroll
                        for (int q2 = 0; q2 < NQ2; ++q2) Z[m][0][q2] = T(0);
                    slab_contract<NSET, NZ>(slab, 0, tl, t2s, Z);
#pragma unroll
                    for (int m = 0; m < NSET; ++m)
#pragma unroll
                        for (int q1 = 0; q1 < Q; ++q1)
                            if (!BAND || in_band<P>(q1, s1))
#pragma unroll
                                for (int q2 = 0; q2 < NQ2; ++q2)
                                    acc[m][q1][q2] = fma((T)f1s[m][q1 * S + s1], Z[m][0][q2], acc[m][q1][q2]);
                } else {
                    slab_contract<NSET, NZ>(slab, s1, tl, t2s, Z);
                }
            }
            // Banded tiles: output q1 has all its slabs once s1 = q1 + P, so it is finished
            // right away (on the grid also stored), and only P + 1 slab results stay live
            if constexpr (EARLY && !ROWS) {
                if (s1 >= P && t.active) emit_q1<NSET, NZ>(s1 - P, f1, Z, out);
            }
            if constexpr (EARLY && ROWS) {
                if (s1 >= P) {
#pragma unroll
                    for (int m = 0; m < NSET; ++m) {
                        const cptr<FT> f1m = fresh(f1[m]);
#pragma unroll
                        for (int q2 = 0; q2 < NQ2; ++q2) O[m][s1 - P][q2] = final_q1<NSET, NZ>(f1m, s1 - P, q2, Z, m);
                    }
                }
            }
        }
        if constexpr (EARLY && !ROWS) return;
        if constexpr (ROWS) {
            const int pos_last = pos0 + n_s1 - 1;
            if constexpr (RUNNING) {
                store_rows<NSET>(pos_last, [&](int m, int q1, int q2) { return acc[m][q1][q2]; }, out);
            } else if constexpr (EARLY) {
                store_rows<NSET>(pos_last, [&](int m, int q1, int q2) { return O[m][q1][q2]; }, out);
            } else {
                store_rows<NSET>(pos_last, [&](int m, int q1, int q2) {
                    return final_q1<NSET, NZ>(fresh(f1[m]), q1, q2, Z, m);
                }, out);
            }
            return;
        }
        if (t.active) {
            const int64_t N2 = (D == 3) ? sp.N[1] : sp.ld, N3 = (D == 3) ? sp.ld : 1;
            const uint32_t lo = (uint32_t)(t.il * Q + ql);
#pragma unroll
            for (int m = 0; m < NSET; ++m) {
                const cptr<FT> f1m = fresh(f1[m]);
#pragma unroll
                for (int q1 = 0; q1 < Q; ++q1) {
#pragma unroll
                    for (int q2 = 0; q2 < NQ2; ++q2) {
                        T v;
                        if constexpr (RUNNING) {
                            v = acc[m][q1][q2];
                        } else {
                            Acc<T, FINAL> a;
#pragma unroll
                            for (int s1 = 0; s1 < S; ++s1)
                                if (!BAND || in_band<P>(q1, s1)) a.add(f1m[q1 * S + s1], fin(Z[m][s1][q2]));
                            v = a.get();
                        }
                        int64_t off;     // wave-uniform part; the lane adds il * Q + ql
                        if constexpr (D == 3) off = ((t.i1 * Q + q1) * N2 + t.i2 * Q + q2) * N3;
                        else off = (t.i1 * Q + q1) * N2;
                        (out[m] + off)[lo] = v;
                    }
                }
            }
        }
    }
};

template <typename T, int P, int D, int WHAT, int FINAL, bool BAND, int WPB, int R, int RING, bool LB, bool ROWS>
__device__ __forceinline__ void adjoint_body(const DevSpace &sp, const DevTabs &tb, const Tile &t, uint32_t *ring,
                                             int lane, const T *__restrict__ gM, const T *__restrict__ gK,
                                             T *__restrict__ dc, T *__restrict__ da0, T *__restrict__ da1,
                                             T *__restrict__ da2) {
    using A = Adjoint<T, P, D, FINAL, BAND, WPB, R, RING, LB, ROWS>;
    constexpr int Q = A::Q, S = A::S, NT = A::NT;
    using FT = typename A::FT;
    constexpr bool DO_M = (WHAT & kWhatM) != 0, DO_K = (WHAT & kWhatK) != 0;
    const int ql = lane - t.r * Q;
    const int s1_lo = (int)(t.i1 >= P ? 0 : P - t.i1);
    const int s1_hi = (int)(sp.n[0] - 1 - t.i1 + P < S - 1 ? sp.n[0] - 1 - t.i1 + P : S - 1);
    const int n_s1 = s1_hi - s1_lo + 1;
    bool fix = t.t0 < P || t.t0 + t.rows_here + P > t.nl;
    if constexpr (D == 3) fix = fix || t.i2 < P || t.i2 >= sp.n[1] - P;
    A adj{sp, t, ring, lane, ql, gM, gK, s1_lo, n_s1, DO_M ? n_s1 : 0, (DO_M ? n_s1 : 0) + (DO_K ? n_s1 : 0), fix};
    adj.make_map();
    const int64_t rs = (int64_t)Q * S;
    cptr<T> M2 = table<T>(tb, 0, 1) + t.i2 * rs;
    cptr<T> K2 = table<T>(tb, 1, 1) + t.i2 * rs;
    const T *ML = (const T *)tb.t[0][D - 1] + t.il * rs + ql * S;
    const T *KL = (const T *)tb.t[1][D - 1] + t.il * rs + ql * S;
    cptr<FT> fM1 = final_table<T, FINAL>(tb, 0, 0) + t.i1 * rs;
    cptr<FT> fK1 = final_table<T, FINAL>(tb, 1, 0) + t.i1 * rs;
    // This lane's last-direction table entries are loaded and consumed before the first
    // slab is issued, so the compiler's wait for them comes before the stream and not
    // inside the slab loop (once a direct-to-LDS load is in flight it can only wait for a
    // register load with a full vmcnt(0); first used under a branch, they would get such a
    // wait at every slab).  The table rows are a few KB shared by every wave: an L2 hit.
    // The first RING - 1 slabs always exist: a row reaches at least p + 1 slabs of each
    // matrix (p + 1 >= 3 >= RING - 1).
    // (banded rows: only the entries s = ql .. ql + P of the lane's node)
    T tlM[NT], tlK[NT];
#pragma unroll
    for (int s = 0; s < NT; ++s) {
        tlM[s] = ML[(LB ? ql : 0) + s];
        tlK[s] = KL[(LB ? ql : 0) + s];
    }
    pin(tlM);
    pin(tlK);
    static_assert(RING - 1 <= P + 1, "prologue slabs exist in every tile");
#pragma unroll
    for (int pos = 0; pos < RING - 1; ++pos) adj.issue(pos);
    if constexpr (DO_M) {
        T tl[1][NT];
#pragma unroll
        for (int s = 0; s < NT; ++s) tl[0][s] = tlM[s];
        const cptr<T> t2[1] = {M2};
        const cptr<FT> f1[1] = {fM1};
        T *const out[1] = {dc};
        adj.template run<1>(0, tl, t2, f1, out);
        phase_barrier();
    }
    if constexpr (DO_K) {
        if constexpr (D == 3) {
            // term 1: (K, M, M), term 2: (M, K, M), term 3: (M, M, K) in directions (1, 2, 3)
            T tl[3][NT];
#pragma unroll
            for (int s = 0; s < NT; ++s) {
                tl[0][s] = tlM[s];
                tl[1][s] = tlM[s];
                tl[2][s] = tlK[s];
            }
            const cptr<T> t2[3] = {M2, K2, M2};
            const cptr<FT> f1[3] = {fK1, fM1, fM1};
            T *const out[3] = {da0, da1, da2};
            adj.template run<3>(adj.nM, tl, t2, f1, out);
        } else {
            // term 1: (K, M), term 2: (M, K) in directions (1, 2)
            T tl[2][NT];
#pragma unroll
            for (int s = 0; s < NT; ++s) {
                tl[0][s] = tlM[s];
                tl[1][s] = tlK[s];
            }
            const cptr<T> t2[2] = {M2, M2};
            const cptr<FT> f1[2] = {fK1, fM1};
            T *const out[2] = {da0, da1};
            adj.template run<2>(adj.nM, tl, t2, f1, out);
        }
    }
}

// Every tile of every line; BANDED: every leading direction's tables are banded, and each
// tile whose leading indices are interior takes the banded loops (the others the full
// loops, which every tile takes when BANDED is false).  One launch for both kinds of tile
// measured faster than a launch per kind (FP32: 2% at 160^3, 4% at 96^3; FP64: 1-12% at
// 160^3), now that both code paths fit the same registers.  ROWS: gradients stored row by
// row.
template <typename T, int P, int D, int WHAT, int FINAL, int WPB, int RING, bool BANDED, bool ROWS>
__global__ __launch_bounds__(64 * WPB) void adjoint_kernel(
    DevSpace sp, DevTabs tb, const T *__restrict__ gM, const T *__restrict__ gK,
    T *__restrict__ dc, T *__restrict__ da0, T *__restrict__ da1, T *__restrict__ da2,
    int64_t task0, int64_t n_tasks, int tiles_per_line) {
    constexpr int Q = P + 1;
    constexpr int R = 64 / Q;                      // rows per wave tile
    using A = Adjoint<T, P, D, FINAL, false, WPB, R, RING, false, ROWS>;
    __shared__ __align__(16) uint32_t ring[WPB][RING * A::SLOT];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));   // uniform per wave
    const int lane = (int)(threadIdx.x & 63);
    // FP32: runs of 8 tiles per XCD, which with 128-byte aligned grid lines measured 2% faster
    // than one contiguous share per XCD (the order FP64 keeps; it helped FP64 by 15% over
    // dispatch order)
    const int64_t task = task0 + (int64_t)(sizeof(T) == 4 ? block_grouped<8>() : block_chunked()) * WPB + wave;
    if (task >= n_tasks) return;
    const Tile t = make_tile<D, P>(sp, task, tiles_per_line, R, Q, lane);
    // banded tiles whose rows are all banded in the last direction too take the short
    // last-direction loops
    const bool last = ((sp.band >> (D - 1)) & 1) && t.t0 >= P && t.t0 + t.rows_here + P <= t.nl;
    if (BANDED && tile_banded<D, P>(sp, t)) {
        if (last)
            adjoint_body<T, P, D, WHAT, FINAL, true, WPB, R, RING, true, ROWS>(sp, tb, t, ring[wave], lane, gM, gK, dc,
                                                                            da0, da1, da2);
        else
            adjoint_body<T, P, D, WHAT, FINAL, true, WPB, R, RING, false, ROWS>(sp, tb, t, ring[wave], lane, gM, gK, dc,
                                                                             da0, da1, da2);
    } else {
        adjoint_body<T, P, D, WHAT, FINAL, false, WPB, R, RING, false, ROWS>(sp, tb, t, ring[wave], lane, gM, gK, dc,
                                                                          da0, da1, da2);
    }
}


// --------------------------------------------------------------------------------------
// Matrix-free products y = M x, y = K x in 2D and the load vector (3D products: the
// blocked kernel of wqa_products.hip).  Lane (r, q_d) as in the adjoint.  The tile's window of x (every column any of its rows reaches: i_k - P ..
// i_k + P in each direction) is staged in LDS, zero outside the space.  Each lane
// contracts the window over s_d, s_{d-1}, ..., s_1 into its node column -- at every point
// of the row, sum_j T(i, q, j) x_j with the product of the directions' tables --
// multiplies by the coefficient samples there and sums over the points; the Q lanes of
// a row add their sums.  Summed over the points this is sum_j M_ij x_j (or K) with the
// same rules, tables and samples as the assembled matrices, which are never stored.
// ONES replaces x by 1 everywhere: by the partition of unity the mass product then
// gives the load vector b_i = integral f B_i with f as the coefficient.
// LB as in Adjoint: the tile's rows are banded in the last direction, so a lane with node
// q_d reads and weighs only the window values s_d = q_d .. q_d + P.
template <typename T, int P, int D, bool BAND, bool ONES, bool LB = false>
struct Apply {
    static constexpr int Q = P + 1, S = 2 * P + 1, R = 64 / Q;
    static constexpr int NT = LB ? P + 1 : S;            // last-direction table entries per lane
    static constexpr int W = R + 2 * P;                  // window length along the last direction
    static constexpr int NQ2 = (D == 3) ? Q : 1;
    static constexpr int NS2 = (D == 3) ? S : 1;

    const DevSpace &sp;
    const Tile &t;
    const T *win;      // this wave's window, [s1][s2][W] (d = 3) or [s1][W]
    int ql;

    // NSET terms that share the window read: term m uses the last-direction table
    // entries tl[ls[m]] (this lane's node ql of row il), the uniform table rows t2[m]
    // (direction 2, d = 3) and t1[m] (direction 1), and the coefficient field f[m].
    // Returns sum_m sum over the lane's points (q1[, q2], ql) of f[m] times the window
    // contracted to that point.
    // PRE: pre holds the coefficient samples of the lane's points (one set), loaded by the
    // caller before the contraction; otherwise they are loaded here at the end.
    template <int NSET, int NL, bool PRE>
    __device__ __forceinline__ T terms(const T *const (&f)[NSET], const cptr<T> (&t1)[NSET],
                                       const cptr<T> (&t2)[NSET], const T (&tl)[NL][NT], const int (&ls)[NSET],
                                       const T (&pre)[Q][NQ2]) const {
        T X[NSET][Q][NQ2];
#pragma unroll
        for (int m = 0; m < NSET; ++m)
#pragma unroll
            for (int q1 = 0; q1 < Q; ++q1)
#pragma unroll
                for (int q2 = 0; q2 < NQ2; ++q2) X[m][q1][q2] = T(0);
        T tsum[NL];
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            tsum[l] = T(0);
            if constexpr (ONES) {
#pragma unroll
                for (int s3 = 0; s3 < NT; ++s3) tsum[l] += tl[l][s3];
            }
        }
        const T *row = win + (t.r < t.rows_here ? t.r : 0) + (LB ? ql : 0);
        // s1 stays a loop: unrolled, the compiler hoists the whole window's reads and holds
        // them in registers (the banded skip over q1 becomes a uniform branch)
#pragma unroll 1
        for (int s1 = 0; s1 < S; ++s1) {
            T Z[NSET][NQ2];
#pragma unroll
            for (int m = 0; m < NSET; ++m)
#pragma unroll
                for (int q2 = 0; q2 < NQ2; ++q2) Z[m][q2] = T(0);
#pragma unroll
            for (int s2 = 0; s2 < NS2; ++s2) {
                // the window row (s1, s2) of this lane's row, contracted over s3 once per
                // last-direction table
                T y[NL];
                if constexpr (ONES) {
#pragma unroll
                    for (int l = 0; l < NL; ++l) y[l] = tsum[l];
                } else {
                    T g[NT];
#pragma unroll
                    for (int s3 = 0; s3 < NT; ++s3) g[s3] = row[(s1 * NS2 + s2) * W + s3];
#pragma unroll
                    for (int l = 0; l < NL; ++l) {
                        y[l] = T(0);
#pragma unroll
                        for (int s3 = 0; s3 < NT; ++s3) y[l] = fma(g[s3], tl[l][s3], y[l]);
                    }
                }
#pragma unroll
                for (int m = 0; m < NSET; ++m) {
                    if constexpr (D == 3) {
#pragma unroll
                        for (int q2 = 0; q2 < Q; ++q2)
                            if (!BAND || in_band<P>(q2, s2)) Z[m][q2] = fma(y[ls[m]], t2[m][q2 * S + s2], Z[m][q2]);
                    } else {
                        Z[m][0] = y[ls[m]];
                    }
                }
            }
#pragma unroll
            for (int m = 0; m < NSET; ++m)
#pragma unroll
                for (int q1 = 0; q1 < Q; ++q1)
                    if (!BAND || in_band<P>(q1, s1))
#pragma unroll
                        for (int q2 = 0; q2 < NQ2; ++q2) X[m][q1][q2] = fma(Z[m][q2], t1[m][q1 * S + s1], X[m][q1][q2]);
        }
        const SampleIndex<D, P> at(sp, t, ql);
        T acc = T(0);
#pragma unroll
        for (int m = 0; m < NSET; ++m)
#pragma unroll
            for (int q1 = 0; q1 < Q; ++q1)
#pragma unroll
                for (int q2 = 0; q2 < NQ2; ++q2) {
                    if constexpr (PRE && NSET == 1) acc = fma(pre[q1][q2], X[m][q1][q2], acc);
                    else acc = fma((f[m] + at.uniform(q1, q2))[at.lo], X[m][q1][q2], acc);
                }
        return acc;
    }
};

template <typename T, int P, int D, int WHAT, bool ONES, bool BAND, bool LB, bool PRE, int NQ2>
__device__ __forceinline__ T apply_body(const DevSpace &sp, const DevTabs &tb, const Tile &t, const T *win, int lane,
                                        const T *__restrict__ cf, const T *__restrict__ a0,
                                        const T *__restrict__ a1, const T *__restrict__ a2,
                                        const T (&pre)[P + 1][NQ2]) {
    using A = Apply<T, P, D, BAND, ONES, LB>;
    constexpr int Q = A::Q, S = A::S, NT = A::NT;
    const int ql = lane - t.r * Q;
    const A ap{sp, t, win, ql};
    const int64_t rs = (int64_t)Q * S;
    cptr<T> M1 = table<T>(tb, 0, 0) + t.i1 * rs, K1 = table<T>(tb, 1, 0) + t.i1 * rs;
    cptr<T> M2 = table<T>(tb, 0, 1) + (D == 3 ? t.i2 : 0) * rs, K2 = table<T>(tb, 1, 1) + (D == 3 ? t.i2 : 0) * rs;
    const T *ML = (const T *)tb.t[0][D - 1] + t.il * rs + ql * S + (LB ? ql : 0);
    const T *KL = (const T *)tb.t[1][D - 1] + t.il * rs + ql * S + (LB ? ql : 0);
    if constexpr (WHAT == kWhatM) {
        T tl[1][NT];
#pragma unroll
        for (int s = 0; s < NT; ++s) tl[0][s] = ML[s];
        const T *const f[1] = {cf};
        const cptr<T> t1[1] = {M1}, t2[1] = {M2};
        const int ls[1] = {0};
        return ap.template terms<1, 1, PRE>(f, t1, t2, tl, ls, pre);
    } else {
        T tl[2][NT];     // mass and stiffness entries of the last direction
#pragma unroll
        for (int s = 0; s < NT; ++s) {
            tl[0][s] = ML[s];
            tl[1][s] = KL[s];
        }
        if constexpr (D == 3) {
            // term k: stiffness table in direction k, mass tables elsewhere
            const T *const f[3] = {a0, a1, a2};
            const cptr<T> t1[3] = {K1, M1, M1}, t2[3] = {M2, K2, M2};
            const int ls[3] = {0, 0, 1};
            return ap.template terms<3, 2, false>(f, t1, t2, tl, ls, pre);
        } else {
            const T *const f[2] = {a0, a1};
            const cptr<T> t1[2] = {K1, M1}, t2[2] = {M2, M2};
            const int ls[2] = {0, 1};
            return ap.template terms<2, 2, false>(f, t1, t2, tl, ls, pre);
        }
    }
}

constexpr int kApplyWaves = 4;      // waves per work-group of apply_kernel

template <typename T, int P, int D, int WHAT, bool ONES>
__global__ __launch_bounds__(64 * kApplyWaves, sizeof(T) == 4 ? 4 : 2) void apply_kernel(DevSpace sp, DevTabs tb, const T *__restrict__ cf,
                                                    const T *__restrict__ a0, const T *__restrict__ a1,
                                                    const T *__restrict__ a2, const T *__restrict__ x,
                                                    T *__restrict__ y, int64_t task0, int64_t n_tasks,
                                                    int tiles_per_line) {
    constexpr int WPB = kApplyWaves, Q = P + 1, S = 2 * P + 1, R = 64 / Q;
    constexpr int W = R + 2 * P, NL = (D == 3) ? S * S : S;
    __shared__ __align__(16) T win[WPB][ONES ? 1 : NL * W];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));   // uniform per wave
    const int lane = (int)(threadIdx.x & 63);
    // XCD-aware order: neighbouring tiles share most of their x windows.  Runs of 8
    // work-groups per XCD measured 2-5% faster than dispatch order (160^3, FP32 and FP64);
    // for FP32 y = K x one contiguous share per XCD did better still (1.19 against 1.25 ms)
    const uint32_t blk = (sizeof(T) == 4 && WHAT == kWhatK && !ONES) ? block_chunked() : block_grouped<8>();
    const int64_t task = task0 + (int64_t)blk * WPB + wave;
    if (task >= n_tasks) return;
    const Tile t = make_tile<D, P>(sp, task, tiles_per_line, R, Q, lane);
    // y = M x in FP64: the coefficient samples of the lane's points are loaded once the window
    // is staged, so that they are in flight while it is contracted (measured in 3D at 160^3,
    // when this kernel served the 3D products: 0.92 against 1.22 ms; 1.01 ms when loaded
    // before the window, whose loads then waited behind them).  In FP32 either made y = M x
    // 30% slower: 16 more registers cost two waves per SIMD there.
    constexpr int NQ2 = (D == 3) ? Q : 1;
    constexpr bool PRE = sizeof(T) == 8 && WHAT == kWhatM && !ONES;
    T pre[Q][NQ2];
    if constexpr (!ONES) {
        // The window is S (d = 3: S x S) lines of W consecutive values of x, one per
        // leading-direction column pair (j_1, j_2).  For each s1 the lanes take the S x W
        // values of its lines, e = s2 W + m (at most NC per lane); their offsets from the
        // line of (j_1, i_2 - P) and their last- and middle-direction ranges are worked out
        // once, so each s1 costs a uniform check of j_1 and NC loads.
        const int64_t n0 = sp.n[0], n1 = (D == 3) ? sp.n[1] : 1, nl = t.nl;
        constexpr int LW = (D == 3) ? S * W : W;          // values per s1
        constexpr int NC = (LW + 63) / 64;
        int64_t off[NC];
        bool ok[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const int e = lane + 64 * k;
            const int s2 = (D == 3) ? e / W : 0, m = e - s2 * W;
            const int64_t j2 = (D == 3) ? t.i2 - P + s2 : 0, j3 = t.t0 - P + m;
            ok[k] = e < LW && j2 >= 0 && j2 < n1 && j3 >= 0 && j3 < nl;
            off[k] = ok[k] ? (j2 - ((D == 3) ? t.i2 - P : 0)) * nl + j3 : 0;
        }
        const int64_t line0 = (D == 3) ? t.i2 - P : 0;     // j_2 of the window's first line
#pragma unroll
        for (int s1 = 0; s1 < S; ++s1) {
            const int64_t j1 = t.i1 - P + s1;
            const bool in = j1 >= 0 && j1 < n0;             // wave-uniform
            const int64_t rowbase = ((in ? j1 : 0) * n1 + line0) * nl;
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                const int e = lane + 64 * k;
                T v = T(0);
                if (in && ok[k]) v = x[rowbase + off[k]];
                if (e < LW) win[wave][s1 * LW + e] = v;
            }
        }
        wave_lds_sync();
    }
    if constexpr (PRE) {
        const SampleIndex<D, P> at(sp, t, lane - t.r * Q);
#pragma unroll
        for (int q1 = 0; q1 < Q; ++q1)
#pragma unroll
            for (int q2 = 0; q2 < NQ2; ++q2) pre[q1][q2] = (cf + at.uniform(q1, q2))[at.lo];
    }
    T v;
    const bool last_banded = ((sp.band >> (D - 1)) & 1) && t.t0 >= P && t.t0 + t.rows_here + P <= t.nl;
    if (tile_banded<D, P>(sp, t)) {
        if (last_banded)
            v = apply_body<T, P, D, WHAT, ONES, true, true, PRE, NQ2>(sp, tb, t, win[wave], lane, cf, a0, a1, a2, pre);
        else
            v = apply_body<T, P, D, WHAT, ONES, true, false, PRE, NQ2>(sp, tb, t, win[wave], lane, cf, a0, a1, a2, pre);
    } else {
        v = apply_body<T, P, D, WHAT, ONES, false, false, PRE, NQ2>(sp, tb, t, win[wave], lane, cf, a0, a1, a2, pre);
    }
    // the row's value is the sum over its Q lanes (lanes r Q .. r Q + Q - 1)
    const int base = t.r * Q;
    T sum = v;
#pragma unroll
    for (int k = 1; k < Q; ++k) sum += __shfl(v, base + k, 64);
    if (t.active && lane == base) y[t.row0 + t.r] = sum;
}

// --- dispatch ----------------------------------------------------------------------------
// Launches kernel(task0, n_tasks) over [0, tasks) in dispatches of at most max_tasks
// tasks (a multiple of wpb), so that no grid passes HIP's 32-bit work-item count.
template <class L>
hipError_t split_launch(int64_t tasks, int64_t max_tasks, int wpb, L launch) {
    const int64_t step = std::max<int64_t>(wpb, max_tasks / wpb * wpb);
    for (int64_t t0 = 0; t0 < tasks; t0 += step) {
        const int64_t here = std::min(step, tasks - t0);
        launch(t0, dim3((unsigned)((here + wpb - 1) / wpb)));
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T, int P, int D, int WHAT, int FINAL>
hipError_t run_forward(const DevSpace &sp, const DevTabs &tb, const void *c, const void *const *a,
                       void *M, void *K, hipStream_t st, int64_t max_tasks) {
    constexpr int S = 2 * P + 1, R = 64 / S;
    // one wave per work-group: the same occupancy as larger groups (set by registers and
    // the whole-tile LDS staging), but finer-grained dispatch; measured 6-9% faster than
    // four waves per group
    constexpr int WPB = 1;
    const int tiles = (int)((sp.n[D - 1] + R - 1) / R);
    int64_t lines = 1;
    for (int k = 0; k < D - 1; ++k) lines *= sp.n[k];
    const int64_t tasks = lines * tiles;
    const T *a0 = nullptr, *a1 = nullptr, *a2 = nullptr;
    if (WHAT & kWhatK) {
        a0 = (const T *)a[0];
        a1 = (const T *)a[1];
        a2 = D == 3 ? (const T *)a[2] : nullptr;
    }
    return split_launch(tasks, max_tasks, WPB, [&](int64_t t0, dim3 grid) {
        const int64_t end = t0 + (int64_t)grid.x * WPB < tasks ? t0 + (int64_t)grid.x * WPB : tasks;
        hipLaunchKernelGGL((forward_kernel<T, P, D, WHAT, FINAL, WPB, R>), grid, dim3(64 * WPB), 0, st, sp, tb,
                           (const T *)c, a0, a1, a2, (T *)M, (T *)K, t0, end, tiles);
    });
}

template <typename T, int P, int D, int WHAT, int FINAL>
hipError_t run_adjoint(const DevSpace &sp, const DevTabs &tb, const void *gM, const void *gK,
                       void *dc, void *const *da, hipStream_t st, int64_t max_tasks) {
    constexpr int Q = P + 1, R = 64 / Q;
    // ring depth: FP32 4 slabs, FP64 3 slabs (a 2-slab ring measured 1.5% slower in FP32);
    // one wave per work-group (as fast as four in FP32, 10% faster than two in FP64)
    constexpr int RING = sizeof(T) == 4 ? 4 : 3;
    constexpr int WPB = 1;
    const int tiles = (int)((sp.n[D - 1] + R - 1) / R);
    int64_t lines = 1;
    for (int k = 0; k < D - 1; ++k) lines *= sp.n[k];
    const int64_t tasks = lines * tiles;
    const int lead = (1 << (D - 1)) - 1;
    const bool banded = (sp.band & lead) == lead;
    T *d0 = nullptr, *d1 = nullptr, *d2 = nullptr;
    if (WHAT & kWhatK) {
        d0 = (T *)da[0];
        d1 = (T *)da[1];
        d2 = D == 3 ? (T *)da[2] : nullptr;
    }
    const dim3 block(64 * WPB);
    return split_launch(tasks, max_tasks, WPB, [&](int64_t t0, dim3 grid) {
        const int64_t end = t0 + (int64_t)grid.x * WPB < tasks ? t0 + (int64_t)grid.x * WPB : tasks;
        auto go = [&](auto kernel) {
            hipLaunchKernelGGL(kernel, grid, block, 0, st, sp, tb, (const T *)gM, (const T *)gK, (T *)dc, d0, d1, d2,
                               t0, end, tiles);
        };
        if (banded) {
            if (sp.rows) go(adjoint_kernel<T, P, D, WHAT, FINAL, WPB, RING, true, true>);
            else go(adjoint_kernel<T, P, D, WHAT, FINAL, WPB, RING, true, false>);
        } else {
            if (sp.rows) go(adjoint_kernel<T, P, D, WHAT, FINAL, WPB, RING, false, true>);
            else go(adjoint_kernel<T, P, D, WHAT, FINAL, WPB, RING, false, false>);
        }
    });
}

template <typename T, int P, int D, int WHAT, bool ONES>
hipError_t run_apply(const DevSpace &sp, const DevTabs &tb, const void *c, const void *const *a, const void *x,
                     void *y, hipStream_t st, int64_t max_tasks) {
    constexpr int Q = P + 1, R = 64 / Q, WPB = kApplyWaves;
    const int tiles = (int)((sp.n[D - 1] + R - 1) / R);
    int64_t lines = 1;
    for (int k = 0; k < D - 1; ++k) lines *= sp.n[k];
    const int64_t tasks = lines * tiles;
    const T *a0 = nullptr, *a1 = nullptr, *a2 = nullptr;
    if (WHAT == kWhatK) {
        a0 = (const T *)a[0];
        a1 = (const T *)a[1];
        a2 = D == 3 ? (const T *)a[2] : nullptr;
    }
    return split_launch(tasks, max_tasks, WPB, [&](int64_t t0, dim3 grid) {
        const int64_t end = t0 + (int64_t)grid.x * WPB < tasks ? t0 + (int64_t)grid.x * WPB : tasks;
        hipLaunchKernelGGL((apply_kernel<T, P, D, WHAT, ONES>), grid, dim3(64 * WPB), 0, st, sp, tb, (const T *)c,
                           a0, a1, a2, (const T *)x, (T *)y, t0, end, tiles);
    });
}

template <typename T, int P, int D>
hipError_t apply_what(int what, bool ones, const DevSpace &sp, const DevTabs &tb, const void *c,
                      const void *const *a, const void *x, void *y, hipStream_t st, int64_t max_tasks) {
    if (ones) return run_apply<T, P, D, kWhatM, true>(sp, tb, c, a, x, y, st, max_tasks);
    if constexpr (D == 3) {
        return hipErrorInvalidValue;              // the 3D products run launch_apply_blocked
    } else {
        if (what == kWhatM) return run_apply<T, P, D, kWhatM, false>(sp, tb, c, a, x, y, st, max_tasks);
        return run_apply<T, P, D, kWhatK, false>(sp, tb, c, a, x, y, st, max_tasks);
    }
}

template <typename T>
hipError_t apply_shape(int what, bool ones, const DevSpace &sp, const DevTabs &tb, const void *c,
                       const void *const *a, const void *x, void *y, hipStream_t st, int64_t max_tasks) {
    if (sp.p == 2 && sp.d == 2) return apply_what<T, 2, 2>(what, ones, sp, tb, c, a, x, y, st, max_tasks);
    if (sp.p == 2 && sp.d == 3) return apply_what<T, 2, 3>(what, ones, sp, tb, c, a, x, y, st, max_tasks);
    if (sp.p == 3 && sp.d == 2) return apply_what<T, 3, 2>(what, ones, sp, tb, c, a, x, y, st, max_tasks);
    if (sp.p == 3 && sp.d == 3) return apply_what<T, 3, 3>(what, ones, sp, tb, c, a, x, y, st, max_tasks);
    return hipErrorInvalidValue;
}

template <typename T, int P, int D, int WHAT>
hipError_t fwd_final(int final_mode, const DevSpace &sp, const DevTabs &tb, const void *c,
                     const void *const *a, void *M, void *K, hipStream_t st, int64_t max_tasks) {
    if constexpr (sizeof(T) == 8) {
        return run_forward<T, P, D, WHAT, 0>(sp, tb, c, a, M, K, st, max_tasks);
    } else {
        switch (final_mode) {
            case 0: return run_forward<T, P, D, WHAT, 0>(sp, tb, c, a, M, K, st, max_tasks);
            case 1: return run_forward<T, P, D, WHAT, 1>(sp, tb, c, a, M, K, st, max_tasks);
            default: return run_forward<T, P, D, WHAT, 2>(sp, tb, c, a, M, K, st, max_tasks);
        }
    }
}

template <typename T, int P, int D, int WHAT>
hipError_t adj_final(int final_mode, const DevSpace &sp, const DevTabs &tb, const void *gM,
                     const void *gK, void *dc, void *const *da, hipStream_t st, int64_t max_tasks) {
    if constexpr (sizeof(T) == 8) {
        return run_adjoint<T, P, D, WHAT, 0>(sp, tb, gM, gK, dc, da, st, max_tasks);
    } else {
        switch (final_mode) {
            case 0: return run_adjoint<T, P, D, WHAT, 0>(sp, tb, gM, gK, dc, da, st, max_tasks);
            case 1: return run_adjoint<T, P, D, WHAT, 1>(sp, tb, gM, gK, dc, da, st, max_tasks);
            default: return run_adjoint<T, P, D, WHAT, 2>(sp, tb, gM, gK, dc, da, st, max_tasks);
        }
    }
}

template <typename T, int P, int D>
hipError_t fwd_what(int final_mode, int what, const DevSpace &sp, const DevTabs &tb, const void *c,
                    const void *const *a, void *M, void *K, hipStream_t st, int64_t max_tasks) {
    switch (what) {
        case kWhatM: return fwd_final<T, P, D, kWhatM>(final_mode, sp, tb, c, a, M, K, st, max_tasks);
        case kWhatK: return fwd_final<T, P, D, kWhatK>(final_mode, sp, tb, c, a, M, K, st, max_tasks);
        default: return fwd_final<T, P, D, kWhatMK>(final_mode, sp, tb, c, a, M, K, st, max_tasks);
    }
}

template <typename T, int P, int D>
hipError_t adj_what(int final_mode, int what, const DevSpace &sp, const DevTabs &tb, const void *gM,
                    const void *gK, void *dc, void *const *da, hipStream_t st, int64_t max_tasks) {
    switch (what) {
        case kWhatM: return adj_final<T, P, D, kWhatM>(final_mode, sp, tb, gM, gK, dc, da, st, max_tasks);
        case kWhatK: return adj_final<T, P, D, kWhatK>(final_mode, sp, tb, gM, gK, dc, da, st, max_tasks);
        default: return adj_final<T, P, D, kWhatMK>(final_mode, sp, tb, gM, gK, dc, da, st, max_tasks);
    }
}

template <typename T>
hipError_t fwd_shape(int final_mode, int what, const DevSpace &sp, const DevTabs &tb, const void *c,
                     const void *const *a, void *M, void *K, hipStream_t st, int64_t max_tasks) {
    if (sp.p == 2 && sp.d == 2) return fwd_what<T, 2, 2>(final_mode, what, sp, tb, c, a, M, K, st, max_tasks);
    if (sp.p == 2 && sp.d == 3) return fwd_what<T, 2, 3>(final_mode, what, sp, tb, c, a, M, K, st, max_tasks);
    if (sp.p == 3 && sp.d == 2) return fwd_what<T, 3, 2>(final_mode, what, sp, tb, c, a, M, K, st, max_tasks);
    if (sp.p == 3 && sp.d == 3) return fwd_what<T, 3, 3>(final_mode, what, sp, tb, c, a, M, K, st, max_tasks);
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t adj_shape(int final_mode, int what, const DevSpace &sp, const DevTabs &tb, const void *gM,
                     const void *gK, void *dc, void *const *da, hipStream_t st, int64_t max_tasks) {
    if (sp.p == 2 && sp.d == 2) return adj_what<T, 2, 2>(final_mode, what, sp, tb, gM, gK, dc, da, st, max_tasks);
    if (sp.p == 2 && sp.d == 3) return adj_what<T, 2, 3>(final_mode, what, sp, tb, gM, gK, dc, da, st, max_tasks);
    if (sp.p == 3 && sp.d == 2) return adj_what<T, 3, 2>(final_mode, what, sp, tb, gM, gK, dc, da, st, max_tasks);
    if (sp.p == 3 && sp.d == 3) return adj_what<T, 3, 3>(final_mode, what, sp, tb, gM, gK, dc, da, st, max_tasks);
    return hipErrorInvalidValue;
}

}  // namespace

// The file is compiled once per part (WQA_PART 0 to 3: forward, products, FP32 adjoint,
// FP64 adjoint), so that the sets of kernels build in parallel.
#if !defined(WQA_PART) || WQA_PART == 0
hipError_t launch_forward(int dtype, int final_mode, int what, const DevSpace &sp, const DevTabs &tb,
                          const void *c, const void *const *a, void *M, void *K, hipStream_t stream,
                          int64_t max_tasks) {
    if (dtype == 0) return fwd_shape<float>(final_mode, what, sp, tb, c, a, M, K, stream, max_tasks);
    return fwd_shape<double>(final_mode, what, sp, tb, c, a, M, K, stream, max_tasks);
}
#endif

#if !defined(WQA_PART) || WQA_PART == 1
hipError_t launch_apply(int dtype, int what, bool ones, const DevSpace &sp, const DevTabs &tb, const void *c,
                        const void *const *a, const void *x, void *y, hipStream_t stream, int64_t max_tasks) {
    if (dtype == 0) return apply_shape<float>(what, ones, sp, tb, c, a, x, y, stream, max_tasks);
    return apply_shape<double>(what, ones, sp, tb, c, a, x, y, stream, max_tasks);
}
#endif

// the adjoint's FP32 and FP64 kernels in parts of their own (WQA_PART 2 and 3)
hipError_t launch_adjoint_f64(int final_mode, int what, const DevSpace &sp, const DevTabs &tb, const void *gM,
                              const void *gK, void *dc, void *const *da, hipStream_t stream, int64_t max_tasks);

#if !defined(WQA_PART) || WQA_PART == 2
hipError_t launch_adjoint(int dtype, int final_mode, int what, const DevSpace &sp, const DevTabs &tb,
                          const void *gM, const void *gK, void *dc, void *const *da, hipStream_t stream,
                          int64_t max_tasks) {
    if (dtype == 0) return adj_shape<float>(final_mode, what, sp, tb, gM, gK, dc, da, stream, max_tasks);
    return launch_adjoint_f64(final_mode, what, sp, tb, gM, gK, dc, da, stream, max_tasks);
}
#endif

#if !defined(WQA_PART) || WQA_PART == 3
hipError_t launch_adjoint_f64(int final_mode, int what, const DevSpace &sp, const DevTabs &tb, const void *gM,
                              const void *gK, void *dc, void *const *da, hipStream_t stream, int64_t max_tasks) {
    return adj_shape<double>(final_mode, what, sp, tb, gM, gK, dc, da, stream, max_tasks);
}
#endif

}  // namespace wqa
