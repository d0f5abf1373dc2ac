// complex64 instantiations of the batching form, and its helper kernels
#include "batch_kernel.cuh"
#include "kernels.h"

namespace qsim {

namespace {

__global__ __launch_bounds__(256) void k_zero_u32(uint32_t *p, uint64_t words)
{
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < words; i += (uint64_t)gridDim.x * 256)
        p[i] = 0;
}

__global__ __launch_bounds__(256) void k_zero_u64(uint64_t *p, uint64_t words)
{
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < words; i += (uint64_t)gridDim.x * 256)
        p[i] = 0;
}

template <typename R> __global__ void k_set_ones(Cplx<R> *s, const uint64_t *starts, int count)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < count) {
        Cplx<R> one;
        one.x = R(1);
        one.y = R(0);
        s[starts[c]] = one;
    }
}

// out[2c] = sum of z partials, out[2c+1] = sum of norm partials of circuit c,
// added over its tiles in a fixed order
__global__ __launch_bounds__(256) void k_batch_reduce(const double *partials, const uint64_t *part_off,
                                                      const uint32_t *part_cnt, double *out)
{
    __shared__ double rn[256], rz[256];
    const int c = blockIdx.x;
    const uint64_t off = part_off[c];
    const uint32_t cnt = part_cnt[c];
    double n = 0, z = 0;
    for (uint32_t t = threadIdx.x; t < cnt; t += 256) {
        n += partials[2 * (off + t)];
        z += partials[2 * (off + t) + 1];
    }
    rn[threadIdx.x] = n;
    rz[threadIdx.x] = z;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            rn[threadIdx.x] += rn[threadIdx.x + w];
            rz[threadIdx.x] += rz[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[2 * c] = rz[0];
        out[2 * c + 1] = rn[0];
    }
}

}  // namespace

void launch_batch_f32(const BatchArgs &b, int log_r, int log_nt, int grid, hipStream_t st)
{
    launch_batch_t<float>(b, log_r, log_nt, grid, st);
}

void launch_batch_init(void *state, qs_dtype dt, uint64_t total_elems, const uint64_t *starts, int count,
                       hipStream_t st)
{
    const uint64_t words = total_elems * (dt == QS_C64 ? 1 : 2);
    const unsigned g = (unsigned)std::min<uint64_t>((words + 255) / 256, 65536);
    hipLaunchKernelGGL(k_zero_u64, dim3(g ? g : 1), dim3(256), 0, st, reinterpret_cast<uint64_t *>(state), words);
    check_launch("batch zero");
    if (dt == QS_C64)
        hipLaunchKernelGGL(k_set_ones<float>, dim3((count + 255) / 256), dim3(256), 0, st,
                           reinterpret_cast<Cplx<float> *>(state), starts, count);
    else
        hipLaunchKernelGGL(k_set_ones<double>, dim3((count + 255) / 256), dim3(256), 0, st,
                           reinterpret_cast<Cplx<double> *>(state), starts, count);
    check_launch("batch basis");
}

void launch_batch_reduce(const double *partials, const uint64_t *part_off, const uint32_t *part_cnt, int count,
                         double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_batch_reduce, dim3(count), dim3(256), 0, st, partials, part_off, part_cnt, out);
    check_launch("batch reduce");
}

void launch_queue_reset(uint32_t *words, uint64_t n_words, hipStream_t st)
{
    // a fill kernel, not a memset: the launch is recorded into a HIP graph
    const uint64_t blocks = std::min<uint64_t>(1024, (n_words + 255) / 256);
    hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)std::max<uint64_t>(1, blocks)), dim3(256), 0, st, words, n_words);
    check_launch("batch queue reset");
}

void launch_batch_queue_f32(const QueueArgs &q, int grid, hipStream_t st) { launch_batch_queue_t<float>(q, grid, st); }

}  // namespace qsim
