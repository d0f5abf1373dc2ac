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
