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
//   * Forward: lane (r, s_d) owns one slot column s_d of row r.  It contracts its row's
//     Q^d samples over q_d against the table column s_d, then over q_{d-1}, ... in
//     registers, and finally over q_1 (the "final pass", selectable accumulation).
//     Results go through a small LDS buffer, one s_1 slab at a time, so that stores
//     to the [row][S^d] output run over consecutive addresses.
//   * Adjoint: lane (r, q_d) owns one node column of row r.  The upstream gradient is
//     staged through LDS one s_1 slab at a time (coalesced loads, slots outside the
//     space zeroed), contracted over s_d, s_{d-1}, ..., and the gradient of every
//     sample is stored directly (consecutive lanes = consecutive grid points).
//   * Stiffness: term k uses the stiffness table in direction k and mass tables
//     elsewhere.  Forward terms with the mass table in direction 1 share the final
//     pass; adjoint terms with the mass table in direction d share the first pass.
#include "wqa_internal.h"

namespace wqa {
namespace {

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// --- final-pass accumulators -------------------------------------------------------
// FINAL 0: plain fused multiply-add in T.
// FINAL 1: compensated dot product (Ogita, Rump and Oishi's Dot2: error-free
//          products via FMA, error-free sums, errors summed separately) in FP32.
// FINAL 2: FP64 accumulation, table factor taken from the FP64 table.
template <typename T, int FINAL>
struct Acc {
    T s = T(0);
    __device__ __forceinline__ void add(T a, T b) { s = fma(a, b, s); }
    __device__ __forceinline__ T get() const { return s; }
};

template <>
struct Acc<float, 1> {
    float p = 0.f, e = 0.f;
    __device__ __forceinline__ void add(float a, float b) {
        float h = a * b;
        float r = __builtin_fmaf(a, b, -h);
        float t = p + h;
        float z = t - p;
        float q = (p - (t - z)) + (h - z);
        p = t;
        e += q + r;
    }
    __device__ __forceinline__ float get() const { return p + e; }
};

template <>
struct Acc<float, 2> {
    double s = 0.0;
    __device__ __forceinline__ void add(double a, float b) { s = __builtin_fma(a, (double)b, s); }
    __device__ __forceinline__ float get() const { return (float)s; }
};

// Table element type used by the final pass.
template <typename T, int FINAL> struct FinalTab { using type = T; };
template <> struct FinalTab<float, 2> { using type = double; };

template <typename T, int FINAL>
__device__ __forceinline__ const typename FinalTab<T, FINAL>::type *final_table(const DevTabs &tb, int kind, int dir) {
    if constexpr (FINAL == 2 && sizeof(T) == 4) return tb.t64[kind][dir];
    else return (const T *)tb.t[kind][dir];
}

// --------------------------------------------------------------------------------------
template <typename T, int P, int D, int WHAT, int FINAL, int WPB>
__global__ __launch_bounds__(64 * WPB) void forward_kernel(
    DevSpace sp, DevTabs tb, const T *__restrict__ cf, const T *__restrict__ a0,
    const T *__restrict__ a1, const T *__restrict__ a2, T *__restrict__ Mo,
    T *__restrict__ Ko, int64_t n_tasks, int tiles_per_line) {
    constexpr int Q = P + 1, S = 2 * P + 1;
    constexpr int R = 64 / S;                     // rows per wave tile
    constexpr int SL = (D == 3) ? S * S : S;      // slots of one s_1 slab
    constexpr int SD = S * SL;
    constexpr bool DO_M = (WHAT & kWhatM) != 0, DO_K = (WHAT & kWhatK) != 0;
    constexpr int NMAT = (DO_M ? 1 : 0) + (DO_K ? 1 : 0);
    using FT = typename FinalTab<T, FINAL>::type;
    __shared__ T stage[WPB][NMAT][R * SL];

    const int wave = (int)(threadIdx.x >> 6);
    const int lane = (int)(threadIdx.x & 63);
    const int64_t task = (int64_t)blockIdx.x * WPB + wave;
    if (task >= n_tasks) return;                  // whole wave leaves; no block barriers below
    const int64_t line = task / tiles_per_line;
    const int tile = (int)(task - line * tiles_per_line);
    const int64_t nl = sp.n[D - 1];
    int64_t i1, i2 = 0;
    if constexpr (D == 3) {
        i1 = line / sp.n[1];
        i2 = line - i1 * sp.n[1];
    } else {
        i1 = line;
    }
    const int64_t t0 = (int64_t)tile * R;
    const int rows_here = (int)((nl - t0) < R ? (nl - t0) : R);
    const int r = lane / S, sl = lane - (lane / S) * S;
    const bool in_tile = r < R;
    const bool active = r < rows_here;
    const int64_t il = t0 + (active ? r : 0);
    const int64_t row0 = line * nl + t0;

    // grid offset of this row's point (q1, [q2,] 0)
    const int64_t N2 = sp.N[1], N3 = (D == 3) ? sp.N[2] : 1;
    int64_t base;
    if constexpr (D == 3) base = ((i1 * Q) * N2 + i2 * Q) * N3 + il * Q;
    else base = (i1 * Q) * N2 + il * Q;

    // table rows: leading directions uniform, last direction per lane
    const T *tM[3], *tK[3];
    const FT *fM1 = final_table<T, FINAL>(tb, 0, 0) + i1 * Q * S;
    const FT *fK1 = final_table<T, FINAL>(tb, 1, 0) + i1 * Q * S;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const int64_t ik = (k == 0) ? i1 : (k == D - 1 ? il : i2);
        tM[k] = (const T *)tb.t[0][k] + ik * Q * S;
        tK[k] = (const T *)tb.t[1][k] + ik * Q * S;
    }
    const bool col_ok_last = (il - P + sl >= 0) && (il - P + sl < nl);

    if constexpr (D == 3) {
        // V[s2][q1] for each needed set; M: c; K: term 1 (a0) and terms 2+3 (a1 + a2)
        T Vm[S][Q], V1[S][Q], V23[S][Q];
        auto contract = [&](const T *__restrict__ f, const T *t3, const T *t2, T (&V)[S][Q], bool accumulate) {
            T tl[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) tl[q] = t3[q * S + sl];
            T U[Q][Q];
#pragma unroll
            for (int q1 = 0; q1 < Q; ++q1)
#pragma unroll
                for (int q2 = 0; q2 < Q; ++q2) {
                    const T *src = f + base + ((int64_t)q1 * N2 + q2) * N3;
                    T acc = T(0);
#pragma unroll
                    for (int q3 = 0; q3 < Q; ++q3) acc = fma(src[q3], tl[q3], acc);
                    U[q1][q2] = acc;
                }
#pragma unroll
            for (int s2 = 0; s2 < S; ++s2)
#pragma unroll
                for (int q1 = 0; q1 < Q; ++q1) {
                    T acc = accumulate ? V[s2][q1] : T(0);
#pragma unroll
                    for (int q2 = 0; q2 < Q; ++q2) acc = fma(U[q1][q2], t2[q2 * S + s2], acc);
                    V[s2][q1] = acc;
                }
        };
        if constexpr (DO_M) contract(cf, tM[2], tM[1], Vm, false);
        if constexpr (DO_K) {
            contract(a0, tM[2], tM[1], V1, false);     // term 1: K table in direction 1 (final pass)
            contract(a1, tM[2], tK[1], V23, false);    // term 2: K table in direction 2
            contract(a2, tK[2], tM[1], V23, true);     // term 3: K table in direction 3
        }
#pragma unroll
        for (int s1 = 0; s1 < S; ++s1) {
            const bool ok1 = (i1 - P + s1 >= 0) && (i1 - P + s1 < sp.n[0]);
            if (in_tile) {
#pragma unroll
                for (int s2 = 0; s2 < S; ++s2) {
                    const bool ok = ok1 && col_ok_last && (i2 - P + s2 >= 0) && (i2 - P + s2 < sp.n[1]);
                    int m = 0;
                    if constexpr (DO_M) {
                        Acc<T, FINAL> acc;
#pragma unroll
                        for (int q1 = 0; q1 < Q; ++q1) acc.add(fM1[q1 * S + s1], Vm[s2][q1]);
                        stage[wave][m][r * SL + s2 * S + sl] = ok ? acc.get() : T(0);
                        ++m;
                    }
                    if constexpr (DO_K) {
                        Acc<T, FINAL> acc;
#pragma unroll
                        for (int q1 = 0; q1 < Q; ++q1) {
                            acc.add(fK1[q1 * S + s1], V1[s2][q1]);
                            acc.add(fM1[q1 * S + s1], V23[s2][q1]);
                        }
                        stage[wave][m][r * SL + s2 * S + sl] = ok ? acc.get() : T(0);
                    }
                }
            }
            wave_lds_sync();
            for (int e = lane; e < rows_here * SL; e += 64) {
                const int rr = e / SL, t = e - (e / SL) * SL;
                const int64_t off = (row0 + rr) * SD + s1 * SL + t;
                int m = 0;
                if constexpr (DO_M) { Mo[off] = stage[wave][m][e]; ++m; }
                if constexpr (DO_K) Ko[off] = stage[wave][m][e];
            }
            wave_lds_sync();
        }
    } else {
        T Um[Q], U1[Q], U2[Q];
        auto contract = [&](const T *__restrict__ f, const T *t2, T (&U)[Q]) {
            T tl[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) tl[q] = t2[q * S + sl];
#pragma unroll
            for (int q1 = 0; q1 < Q; ++q1) {
                const T *src = f + base + (int64_t)q1 * N2;
                T acc = T(0);
#pragma unroll
                for (int q2 = 0; q2 < Q; ++q2) acc = fma(src[q2], tl[q2], acc);
                U[q1] = acc;
            }
        };
        if constexpr (DO_M) contract(cf, tM[1], Um);
        if constexpr (DO_K) {
            contract(a0, tM[1], U1);   // term 1: K table in direction 1 (final pass)
            contract(a1, tK[1], U2);   // term 2: K table in direction 2
        }
#pragma unroll
        for (int s1 = 0; s1 < S; ++s1) {
            const bool ok = col_ok_last && (i1 - P + s1 >= 0) && (i1 - P + s1 < sp.n[0]);
            if (in_tile) {
                int m = 0;
                if constexpr (DO_M) {
                    Acc<T, FINAL> acc;
#pragma unroll
                    for (int q1 = 0; q1 < Q; ++q1) acc.add(fM1[q1 * S + s1], Um[q1]);
                    stage[wave][m][r * SL + sl] = ok ? acc.get() : T(0);
                    ++m;
                }
                if constexpr (DO_K) {
                    Acc<T, FINAL> acc;
#pragma unroll
                    for (int q1 = 0; q1 < Q; ++q1) {
                        acc.add(fK1[q1 * S + s1], U1[q1]);
                        acc.add(fM1[q1 * S + s1], U2[q1]);
                    }
                    stage[wave][m][r * SL + sl] = ok ? acc.get() : T(0);
                }
            }
            wave_lds_sync();
            for (int e = lane; e < rows_here * SL; e += 64) {
                const int rr = e / SL, t = e - (e / SL) * SL;
                const int64_t off = (row0 + rr) * SD + s1 * SL + t;
                int m = 0;
                if constexpr (DO_M) { Mo[off] = stage[wave][m][e]; ++m; }
                if constexpr (DO_K) Ko[off] = stage[wave][m][e];
            }
            wave_lds_sync();
        }
    }
}

// --------------------------------------------------------------------------------------
template <typename T, int P, int D, int WHAT, int FINAL, int WPB>
__global__ __launch_bounds__(64 * WPB) void adjoint_kernel(
    DevSpace sp, DevTabs tb, const T *__restrict__ gM, const T *__restrict__ gK,
    T *__restrict__ dc, T *__restrict__ da0, T *__restrict__ da1, T *__restrict__ da2,
    int64_t n_tasks, int tiles_per_line) {
    constexpr int Q = P + 1, S = 2 * P + 1;
    constexpr int R = 64 / Q;                     // rows per wave tile
    constexpr int SL = (D == 3) ? S * S : S;
    constexpr int SD = S * SL;
    constexpr bool DO_M = (WHAT & kWhatM) != 0, DO_K = (WHAT & kWhatK) != 0;
    constexpr int NG = (DO_M ? 1 : 0) + (DO_K ? 1 : 0);
    constexpr int NQ = (D == 3) ? Q * Q : Q;      // outputs per lane per field
    using FT = typename FinalTab<T, FINAL>::type;
    __shared__ T stage[WPB][NG][R * SL];

    const int wave = (int)(threadIdx.x >> 6);
    const int lane = (int)(threadIdx.x & 63);
    const int64_t task = (int64_t)blockIdx.x * WPB + wave;
    if (task >= n_tasks) return;
    const int64_t line = task / tiles_per_line;
    const int tile = (int)(task - line * tiles_per_line);
    const int64_t nl = sp.n[D - 1];
    int64_t i1, i2 = 0;
    if constexpr (D == 3) {
        i1 = line / sp.n[1];
        i2 = line - i1 * sp.n[1];
    } else {
        i1 = line;
    }
    const int64_t t0 = (int64_t)tile * R;
    const int rows_here = (int)((nl - t0) < R ? (nl - t0) : R);
    const int r = lane / Q, ql = lane - (lane / Q) * Q;
    const bool in_tile = r < R;
    const bool active = r < rows_here;
    const int64_t il = t0 + (active ? r : 0);
    const int64_t row0 = line * nl + t0;

    const T *tM[3], *tK[3];
    const FT *fM1 = final_table<T, FINAL>(tb, 0, 0) + i1 * Q * S;
    const FT *fK1 = final_table<T, FINAL>(tb, 1, 0) + i1 * Q * S;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const int64_t ik = (k == 0) ? i1 : (k == D - 1 ? il : i2);
        tM[k] = (const T *)tb.t[0][k] + ik * Q * S;
        tK[k] = (const T *)tb.t[1][k] + ik * Q * S;
    }
    // this lane's node column of the last-direction tables
    T tlM[S], tlK[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        tlM[s] = tM[D - 1][ql * S + s];
        tlK[s] = DO_K ? tK[D - 1][ql * S + s] : T(0);
    }

    // accumulators over s_1: index q1 * (D == 3 ? Q : 1) + q2
    Acc<T, FINAL> accM[DO_M ? NQ : 1];
    Acc<T, FINAL> accK[DO_K ? D : 1][DO_K ? NQ : 1];

    for (int s1 = 0; s1 < S; ++s1) {
        if (i1 - P + s1 < 0 || i1 - P + s1 >= sp.n[0]) continue;   // whole slab outside: zero
        // stage the s1 slab of every row of the tile, slots outside the space zeroed
        for (int e = lane; e < rows_here * SL; e += 64) {
            const int rr = e / SL, t = e - (e / SL) * SL;
            bool ok;
            if constexpr (D == 3) {
                const int64_t j2 = i2 - P + t / S, j3 = t0 + rr - P + t % S;
                ok = j2 >= 0 && j2 < sp.n[1] && j3 >= 0 && j3 < nl;
            } else {
                const int64_t j2 = t0 + rr - P + t;
                ok = j2 >= 0 && j2 < nl;
            }
            const int64_t off = (row0 + rr) * SD + (int64_t)s1 * SL + t;
            int g = 0;
            if constexpr (DO_M) { stage[wave][g][e] = ok ? gM[off] : T(0); ++g; }
            if constexpr (DO_K) stage[wave][g][e] = ok ? gK[off] : T(0);
        }
        wave_lds_sync();
        if (in_tile) {
            const int rb = (r < rows_here ? r : 0) * SL;
            if constexpr (D == 3) {
                T Zm[Q], Z1[Q], Z2[Q], Z3[Q];
#pragma unroll
                for (int q = 0; q < Q; ++q) Zm[q] = Z1[q] = Z2[q] = Z3[q] = T(0);
#pragma unroll
                for (int s2 = 0; s2 < S; ++s2) {
                    if constexpr (DO_M) {
                        const T *g = &stage[wave][0][rb + s2 * S];
                        T y = T(0);
#pragma unroll
                        for (int s3 = 0; s3 < S; ++s3) y = fma(g[s3], tlM[s3], y);
#pragma unroll
                        for (int q2 = 0; q2 < Q; ++q2) Zm[q2] = fma(y, tM[1][q2 * S + s2], Zm[q2]);
                    }
                    if constexpr (DO_K) {
                        const T *g = &stage[wave][DO_M ? 1 : 0][rb + s2 * S];
                        T y12 = T(0), y3 = T(0);
#pragma unroll
                        for (int s3 = 0; s3 < S; ++s3) {
                            y12 = fma(g[s3], tlM[s3], y12);
                            y3 = fma(g[s3], tlK[s3], y3);
                        }
#pragma unroll
                        for (int q2 = 0; q2 < Q; ++q2) {
                            Z1[q2] = fma(y12, tM[1][q2 * S + s2], Z1[q2]);
                            Z2[q2] = fma(y12, tK[1][q2 * S + s2], Z2[q2]);
                            Z3[q2] = fma(y3, tM[1][q2 * S + s2], Z3[q2]);
                        }
                    }
                }
#pragma unroll
                for (int q1 = 0; q1 < Q; ++q1)
#pragma unroll
                    for (int q2 = 0; q2 < Q; ++q2) {
                        if constexpr (DO_M) accM[q1 * Q + q2].add(fM1[q1 * S + s1], Zm[q2]);
                        if constexpr (DO_K) {
                            accK[0][q1 * Q + q2].add(fK1[q1 * S + s1], Z1[q2]);
                            accK[1][q1 * Q + q2].add(fM1[q1 * S + s1], Z2[q2]);
                            accK[2][q1 * Q + q2].add(fM1[q1 * S + s1], Z3[q2]);
                        }
                    }
            } else {
                if constexpr (DO_M) {
                    const T *g = &stage[wave][0][rb];
                    T y = T(0);
#pragma unroll
                    for (int s2 = 0; s2 < S; ++s2) y = fma(g[s2], tlM[s2], y);
#pragma unroll
                    for (int q1 = 0; q1 < Q; ++q1) accM[q1].add(fM1[q1 * S + s1], y);
                }
                if constexpr (DO_K) {
                    const T *g = &stage[wave][DO_M ? 1 : 0][rb];
                    T y1 = T(0), y2 = T(0);
#pragma unroll
                    for (int s2 = 0; s2 < S; ++s2) {
                        y1 = fma(g[s2], tlM[s2], y1);
                        y2 = fma(g[s2], tlK[s2], y2);
                    }
#pragma unroll
                    for (int q1 = 0; q1 < Q; ++q1) {
                        accK[0][q1].add(fK1[q1 * S + s1], y1);
                        accK[1][q1].add(fM1[q1 * S + s1], y2);
                    }
                }
            }
        }
        wave_lds_sync();
    }

    if (!active) return;
    const int64_t N2 = sp.N[1], N3 = (D == 3) ? sp.N[2] : 1;
#pragma unroll
    for (int q1 = 0; q1 < Q; ++q1) {
        if constexpr (D == 3) {
#pragma unroll
            for (int q2 = 0; q2 < Q; ++q2) {
                const int64_t off = ((i1 * Q + q1) * N2 + i2 * Q + q2) * N3 + il * Q + ql;
                if constexpr (DO_M) dc[off] = accM[q1 * Q + q2].get();
                if constexpr (DO_K) {
                    da0[off] = accK[0][q1 * Q + q2].get();
                    da1[off] = accK[1][q1 * Q + q2].get();
                    da2[off] = accK[2][q1 * Q + q2].get();
                }
            }
        } else {
            const int64_t off = (i1 * Q + q1) * N2 + il * Q + ql;
            if constexpr (DO_M) dc[off] = accM[q1].get();
            if constexpr (DO_K) {
                da0[off] = accK[0][q1].get();
                da1[off] = accK[1][q1].get();
            }
        }
    }
}

// --- dispatch ----------------------------------------------------------------------------
constexpr int kWavesPerBlock = 4;

template <typename T, int P, int D, int WHAT, int FINAL>
hipError_t run_forward(const DevSpace &sp, const DevTabs &tb, const void *c, const void *const *a,
                       void *M, void *K, hipStream_t st) {
    constexpr int S = 2 * P + 1, R = 64 / S;
    const int64_t nl = sp.n[D - 1];
    const int tiles = (int)((nl + R - 1) / R);
    int64_t lines = 1;
    for (int k = 0; k < D - 1; ++k) lines *= sp.n[k];
    const int64_t tasks = lines * tiles;
    const int64_t blocks = (tasks + kWavesPerBlock - 1) / kWavesPerBlock;
    const T *a0 = nullptr, *a1 = nullptr, *a2 = nullptr;
    if (WHAT & kWhatK) {
        a0 = (const T *)a[0];
        a1 = (const T *)a[1];
        a2 = D == 3 ? (const T *)a[2] : nullptr;
    }
    hipLaunchKernelGGL((forward_kernel<T, P, D, WHAT, FINAL, kWavesPerBlock>), dim3((unsigned)blocks),
                       dim3(64 * kWavesPerBlock), 0, st, sp, tb, (const T *)c, a0, a1, a2, (T *)M,
                       (T *)K, tasks, tiles);
    return hipGetLastError();
}

template <typename T, int P, int D, int WHAT, int FINAL>
hipError_t run_adjoint(const DevSpace &sp, const DevTabs &tb, const void *gM, const void *gK,
                       void *dc, void *const *da, hipStream_t st) {
    constexpr int Q = P + 1, R = 64 / Q;
    const int64_t nl = sp.n[D - 1];
    const int tiles = (int)((nl + R - 1) / R);
    int64_t lines = 1;
    for (int k = 0; k < D - 1; ++k) lines *= sp.n[k];
    const int64_t tasks = lines * tiles;
    const int64_t blocks = (tasks + kWavesPerBlock - 1) / kWavesPerBlock;
    T *d0 = nullptr, *d1 = nullptr, *d2 = nullptr;
    if (WHAT & kWhatK) {
        d0 = (T *)da[0];
        d1 = (T *)da[1];
        d2 = D == 3 ? (T *)da[2] : nullptr;
    }
    hipLaunchKernelGGL((adjoint_kernel<T, P, D, WHAT, FINAL, kWavesPerBlock>), dim3((unsigned)blocks),
                       dim3(64 * kWavesPerBlock), 0, st, sp, tb, (const T *)gM, (const T *)gK, (T *)dc,
                       d0, d1, d2, tasks, tiles);
    return hipGetLastError();
}

template <typename T, int P, int D, int WHAT>
hipError_t fwd_final(int final_mode, const DevSpace &sp, const DevTabs &tb, const void *c,
                     const void *const *a, void *M, void *K, hipStream_t st) {
    if constexpr (sizeof(T) == 8) {
        return run_forward<T, P, D, WHAT, 0>(sp, tb, c, a, M, K, st);
    } else {
        switch (final_mode) {
            case 0: return run_forward<T, P, D, WHAT, 0>(sp, tb, c, a, M, K, st);
            case 1: return run_forward<T, P, D, WHAT, 1>(sp, tb, c, a, M, K, st);
            default: return run_forward<T, P, D, WHAT, 2>(sp, tb, c, a, M, K, st);
        }
    }
}

template <typename T, int P, int D, int WHAT>
hipError_t adj_final(int final_mode, const DevSpace &sp, const DevTabs &tb, const void *gM,
                     const void *gK, void *dc, void *const *da, hipStream_t st) {
    if constexpr (sizeof(T) == 8) {
        return run_adjoint<T, P, D, WHAT, 0>(sp, tb, gM, gK, dc, da, st);
    } else {
        switch (final_mode) {
            case 0: return run_adjoint<T, P, D, WHAT, 0>(sp, tb, gM, gK, dc, da, st);
            case 1: return run_adjoint<T, P, D, WHAT, 1>(sp, tb, gM, gK, dc, da, st);
            default: return run_adjoint<T, P, D, WHAT, 2>(sp, tb, gM, gK, dc, da, st);
        }
    }
}

template <typename T, int P, int D>
hipError_t fwd_what(int final_mode, int what, const DevSpace &sp, const DevTabs &tb, const void *c,
                    const void *const *a, void *M, void *K, hipStream_t st) {
    switch (what) {
        case kWhatM: return fwd_final<T, P, D, kWhatM>(final_mode, sp, tb, c, a, M, K, st);
        case kWhatK: return fwd_final<T, P, D, kWhatK>(final_mode, sp, tb, c, a, M, K, st);
        default: return fwd_final<T, P, D, kWhatMK>(final_mode, sp, tb, c, a, M, K, st);
    }
}

template <typename T, int P, int D>
hipError_t adj_what(int final_mode, int what, const DevSpace &sp, const DevTabs &tb, const void *gM,
                    const void *gK, void *dc, void *const *da, hipStream_t st) {
    switch (what) {
        case kWhatM: return adj_final<T, P, D, kWhatM>(final_mode, sp, tb, gM, gK, dc, da, st);
        case kWhatK: return adj_final<T, P, D, kWhatK>(final_mode, sp, tb, gM, gK, dc, da, st);
        default: return adj_final<T, P, D, kWhatMK>(final_mode, sp, tb, gM, gK, dc, da, st);
    }
}

template <typename T>
hipError_t fwd_shape(int final_mode, int what, const DevSpace &sp, const DevTabs &tb, const void *c,
                     const void *const *a, void *M, void *K, hipStream_t st) {
    if (sp.p == 2 && sp.d == 2) return fwd_what<T, 2, 2>(final_mode, what, sp, tb, c, a, M, K, st);
    if (sp.p == 2 && sp.d == 3) return fwd_what<T, 2, 3>(final_mode, what, sp, tb, c, a, M, K, st);
    if (sp.p == 3 && sp.d == 2) return fwd_what<T, 3, 2>(final_mode, what, sp, tb, c, a, M, K, st);
    if (sp.p == 3 && sp.d == 3) return fwd_what<T, 3, 3>(final_mode, what, sp, tb, c, a, M, K, st);
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t adj_shape(int final_mode, int what, const DevSpace &sp, const DevTabs &tb, const void *gM,
                     const void *gK, void *dc, void *const *da, hipStream_t st) {
    if (sp.p == 2 && sp.d == 2) return adj_what<T, 2, 2>(final_mode, what, sp, tb, gM, gK, dc, da, st);
    if (sp.p == 2 && sp.d == 3) return adj_what<T, 2, 3>(final_mode, what, sp, tb, gM, gK, dc, da, st);
    if (sp.p == 3 && sp.d == 2) return adj_what<T, 3, 2>(final_mode, what, sp, tb, gM, gK, dc, da, st);
    if (sp.p == 3 && sp.d == 3) return adj_what<T, 3, 3>(final_mode, what, sp, tb, gM, gK, dc, da, st);
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_forward(int dtype, int final_mode, int what, const DevSpace &sp, const DevTabs &tb,
                          const void *c, const void *const *a, void *M, void *K, hipStream_t stream) {
    if (dtype == 0) return fwd_shape<float>(final_mode, what, sp, tb, c, a, M, K, stream);
    return fwd_shape<double>(final_mode, what, sp, tb, c, a, M, K, stream);
}

hipError_t launch_adjoint(int dtype, int final_mode, int what, const DevSpace &sp, const DevTabs &tb,
                          const void *gM, const void *gK, void *dc, void *const *da, hipStream_t stream) {
    if (dtype == 0) return adj_shape<float>(final_mode, what, sp, tb, gM, gK, dc, da, stream);
    return adj_shape<double>(final_mode, what, sp, tb, gM, gK, dc, da, stream);
}

}  // namespace wqa
