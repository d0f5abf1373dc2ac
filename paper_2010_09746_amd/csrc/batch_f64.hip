// complex128 instantiations of the batching form
#include "batch_kernel.cuh"
#include "kernels.h"

namespace qsim {
void launch_batch_f64(const BatchArgs &b, int log_r, int log_nt, int grid, hipStream_t st)
{
    launch_batch_t<double>(b, log_r, log_nt, grid, st);
}

void launch_batch_queue_f64(const QueueArgs &q, int grid, hipStream_t st) { launch_batch_queue_t<double>(q, grid, st); }
}  // namespace qsim
