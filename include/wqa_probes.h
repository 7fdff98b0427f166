/*
 * wqa_probes.h -- memory-pattern probes for libwqa's kernels (libwqa_probes.so).
 *
 * Measurement infrastructure, not part of the assembly library: each probe moves the
 * bytes one of libwqa's kernels moves, in the same order and from the same addresses
 * (same tiles, same work-group order, same kind of load and store instructions), with
 * no arithmetic beyond touching what it loads.  Timed beside the kernel, a probe gives
 * the bandwidth ceiling of that data layout on the GPU at hand.  The plain streaming
 * probes give the ceiling of the simplest patterns.
 *
 * Every buffer is a device pointer owned by the caller, 16-byte aligned; calls are
 * asynchronous on the given HIP stream (NULL = default stream) and return 0, or a
 * negative value for bad arguments (-1) or a launch error (-5).  The probes write
 * their output buffers with meaningless values.
 *
 * Geometry arguments follow libwqa (include/wqa.h): degree p in {2, 3}, d = 3,
 * n_elem[3] elements per direction, rows = prod (n_elem[k] + p), matrices [rows][S^3],
 * grids [N_1][N_2][N_3] with N_k = (n_elem[k] + p)(p + 1).  dtype 0 = FP32, 1 = FP64.
 */
#ifndef WQA_PROBES_H
#define WQA_PROBES_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Plain streaming over n_bytes (a multiple of 16): what = 0 writes dst, 1 reads src
 * (a one-value result goes to dst), 2 copies src to dst.  Each wave moves 1 KB per
 * step with 16-byte accesses, consecutive waves consecutive kilobytes. */
int wqap_stream(int what, void *dst, const void *src, int64_t n_bytes, void *hip_stream);

/* k write fronts: front f is the byte range [f spacing, f spacing + per_front) of dst
 * (per_front a multiple of 4096, spacing >= per_front and a multiple of 16); the waves
 * sweep all fronts at once, each front in 4 KB blocks in address order.  The write rate
 * against k shows what concurrently written regions cost. */
int wqap_fronts(void *dst, int k, int64_t spacing, int64_t per_front, void *hip_stream);

/* The adjoint's pattern: per wave tile of 64/(p+1) consecutive rows of one line, the
 * tile's rows of gM and then gK stream slab by slab (one first-direction slot s_1 at a
 * time) through a ring in LDS filled by direct global-to-LDS loads, and after slab s_1
 * >= p the gradients of node q_1 = s_1 - p are written, one 4- or 8-byte value per lane
 * at consecutive grid points (dc after the gM slabs, da_1..da_3 after the gK slabs).
 * parts: 1 = the loads only, 2 = the stores only, 3 = both.  layout 0 is the kernel's
 * (one wave per work-group, each XCD one contiguous share of the tiles); 1..47 = 16 r +
 * t: work-groups of up to t tiles of one line that stage each (field, q_1) in LDS and
 * write it with 16-byte stores as whole-segment runs, a ring of r + 2 slabs per wave;
 * 48: per tile each matrix's rows loaded into LDS at once, then that matrix's gradients
 * written; 49: the kernel's layout with each matrix's gradients written after its last
 * slab.  Bits 6-7 choose the work-group order (0: each XCD a contiguous share, 1:
 * dispatch order, 2: runs of 8 tiles per XCD); bit 8 (layout 0 only) writes the outputs
 * with grid lines padded to a multiple of 32 values (outputs of N_1 N_2 pitch values, pitch
 * = N_3 rounded up to 32); bit 9 (layout 0 only) stores the gradients row by row
 * ([rows][(p+1)^3], each tile's rows of a field one contiguous block, written with 16-byte
 * stores after each matrix's last slab); bit 10 (p = 3) the same layout written q_1 by q_1
 * as each completes, one 16-byte store per lane (64 bytes per row); bit 11 the same layout
 * after each matrix's last slab with one 4-byte store per lane and (q_1, q_2); bit 12 (layout
 * 0 only) a ring of 3 slabs, whose smaller LDS share lets 16 waves share a CU; bit 13 (layout
 * 0 only) at most 8 waves per CU (each work-group padded to 20 KB of LDS); bit 14 (p = 3) the
 * row-by-row blocks after each matrix's last slab, one 16-byte store per lane and q_1 as a lane
 * (r, j) holds them after a transpose within its quad (64 bytes of row r per store); bit 15 (p = 3)
 * gradients in line-q_1 blocks, [i_1][i_2][q_1][i_3][q_2][q_3]: as each q_1 completes, the
 * tile's values of that q_1 form one contiguous 1 KB block, one 16-byte store per lane.
 * out[4] = dc, da_1, da_2, da_3. */
int wqap_adjoint(int parts, int layout, int dtype, int p, const int64_t *n_elem, const void *gM,
                 const void *gK, void *const *out, void *hip_stream);

/* The forward's pattern: per wave tile of floor(64/(2p+1)) rows, the samples of the
 * four fields (c, a_1..a_3) the tile owns are loaded (16-byte loads where the runs
 * allow), and the tile's rows of M and K are written as two contiguous ranges with
 * 16-byte stores (nontemporal in FP32).  parts: bits 0-1 as above; bits 4-5 the
 * work-group order (0: the kernel's on the grid, runs of 8 consecutive tiles per XCD; 1:
 * each XCD one contiguous share; 2: dispatch order; 3: runs of 128 tiles per XCD, the
 * kernel's with samples stored row by row); bits 6-7: 1 ordinary stores in FP32, 2 M only,
 * 3 every whole 128-byte line the tile's output ranges touch (their end lines shared with
 * the neighbouring tiles, so each tile's stores start and end on line boundaries; the values
 * come from LDS as in the kernel); bit 8: fields with grid lines padded to a multiple of 32
 * values (as for the adjoint); bit 9: fields stored row by row ([rows][(p+1)^3]), each
 * tile's samples of a field one contiguous block loaded with 16-byte loads; bit 10: the
 * 16-byte stores of each range start at its first 128-byte boundary (the values before it
 * take one 4- or 8-byte store per lane), so that each store instruction covers whole lines;
 * bit 11: the 16-byte stores write constants instead of values read from LDS.
 * fields[4] = c, a_1, a_2, a_3; M is needed even for the loads alone. */
int wqap_forward(int parts, int dtype, int p, const int64_t *n_elem, const void *const *fields, void *M,
                 void *K, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* WQA_PROBES_H */
