// Host-side launchers of the HIP kernels (defined in the .hip sources).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "internal.h"

namespace qsim {

// |x> at physical index x; every other amplitude zero.
void launch_set_basis(void *state, qs_dtype dt, int n, uint64_t x, hipStream_t st);

// One gate on physical positions (g.q0, g.q1): the plain form.
void launch_plain_gate(void *state, qs_dtype dt, int n, const qs_gate &g, hipStream_t st);

// In-place data movement: the amplitude at physical index x moves to the
// index whose bit pi[p] is bit p of x.  pi must be an involution.
void launch_involution(void *state, qs_dtype dt, int n, const std::vector<int> &pi, hipStream_t st);

// One fused tile pass.
void launch_tile_f32(const TileArgs &a, uint64_t n_tiles, int log_r, int log_nt, hipStream_t st);
void launch_tile_f64(const TileArgs &a, uint64_t n_tiles, int log_r, int log_nt, hipStream_t st);
// the passes that do not move whole 128-byte lines (plain loads and stores)
void launch_tile_f32_plain(const TileArgs &a, uint64_t n_tiles, int log_r, int log_nt, hipStream_t st);
void launch_tile_f64_plain(const TileArgs &a, uint64_t n_tiles, int log_r, int log_nt, hipStream_t st);
// The same, each tile also writing its per-bit probability sums to zparts
// (1 + log_r + log_nt doubles per tile, see run_range's ZB read-out); passes
// over whole 128-byte lines only (TileArgs::io bit 3).
void launch_tile_f32_z(const TileArgs &a, uint64_t n_tiles, int log_r, int log_nt, double *zparts,
                       hipStream_t st);
void launch_tile_f64_z(const TileArgs &a, uint64_t n_tiles, int log_r, int log_nt, double *zparts,
                       hipStream_t st);

// Batching form.  All states |0> (element offsets of each circuit's first
// amplitude in starts_dev), one persistent launch per pass level, then the
// per-circuit read-out out_dev[2c] = <Z_0>, out_dev[2c+1] = norm.
void launch_batch_init(void *state, qs_dtype dt, uint64_t total_elems, const uint64_t *starts_dev, int count,
                       hipStream_t st);
void launch_batch_f32(const BatchArgs &b, int log_r, int log_nt, int grid, hipStream_t st);
void launch_batch_f64(const BatchArgs &b, int log_r, int log_nt, int grid, hipStream_t st);
void launch_batch_reduce(const double *partials, const uint64_t *part_off, const uint32_t *part_cnt, int count,
                         double *out, hipStream_t st);

// Single-launch batch executor: zero the ticket and the per-pass completion
// counters, then one persistent launch of `grid` workgroups over every work
// item (see QueueArgs).
void launch_queue_reset(uint32_t *words, uint64_t n_words, hipStream_t st);
void launch_batch_queue_f32(const QueueArgs &q, int grid, hipStream_t st);
void launch_batch_queue_f64(const QueueArgs &q, int grid, hipStream_t st);
// largest register bits of a queue item's tile (2^(8 + shape) amplitudes)
constexpr int QUEUE_MIN_SHAPE = 1, QUEUE_MAX_SHAPE = 4, QUEUE_LOG_NT = 8;

// Read-out: norm and position sums S_p = sum_j |v_j|^2 bit_p(j), written to
// out_dev[0] (norm) and out_dev[1 + p].  work_dev holds the block partials.
size_t zsum_work_doubles(int n);
void launch_zsum(const void *state, qs_dtype dt, int n, double *work_dev, double *out_dev,
                 hipStream_t st);

// The same sums from the per-tile read-out of a tile pass (zparts of
// launch_tile_f32_z/f64_z, nv values per tile, value v of tile t at
// parts[v * tiles + t]: T, then B_v for v = 1..nv-1, the bits of the pass's
// store layout, slot bits first).  Output 1 + p sums,
// over tiles t, the probability that bit p is 1 where that bit is the XOR of
// the layout bit v[p] (none when v[p] < 1) and of the bits of the tile index
// in rm[p]: B_v or T - B_v by the parity of t & rm[p], or T or 0 without a
// layout bit.  (Bit p of the state after a pass and some CNOTs is such an
// XOR of bits before them.)
struct ZFoldMap {
    int32_t v[64];
    uint64_t rm[64];
};
// work_dev: zfold_work_doubles(tiles, n) doubles of partial sums
size_t zfold_work_doubles(uint64_t tiles, int n);
void launch_zfold(const double *parts, uint64_t tiles, int nv, int n, const ZFoldMap &m, double *work_dev,
                  double *out_dev, hipStream_t st);

// out_dev[2i], out_dev[2i+1] = amplitude at physical index idx_dev[i] (FP64).
void launch_gather(const void *state, qs_dtype dt, const uint64_t *idx_dev, int64_t count,
                   double *out_dev, hipStream_t st);

// Overlap of two states of n qubits: b is read at the physical index whose bit
// map_b[p] is bit p of a's index (identity when the placements agree).
// out_dev: [re <a|b>, im <a|b>, <a|a>, <b|b>, max |a - b|].
size_t fid_work_doubles(int n);
void launch_fidelity(const void *a, qs_dtype da, const void *b, qs_dtype db, int n,
                     const std::vector<int> &map_b, double *work_dev, double *out_dev,
                     hipStream_t st);

}  // namespace qsim
