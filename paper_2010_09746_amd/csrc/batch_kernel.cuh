// Batching form: many independent circuits of different sizes, advanced one
// pass level at a time.  A level holds every circuit's tile pass of that index;
// its work items (ranges of tiles) are independent, so one persistent launch
// per level strides over them with no waiting between workgroups, and the
// ordering between a circuit's consecutive passes comes from the launch order.
// The whole sequence of level launches is captured once in a HIP graph.
#pragma once

#include "tile_kernel.cuh"

namespace qsim {

template <typename R, int LOG_NT, int LOG_R>
__global__ __launch_bounds__(1 << LOG_NT) void k_batch(BatchArgs b)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    // whole amplitudes per re-layout round: the persistent grid, not LDS,
    // sets how many workgroups are resident; ordinary (cached) loads and
    // stores: the states are small and are read again at the next level
    using TK = TileKernel<R, LOG_NT, LOG_R, false, false>;
    using PassPtr = const __attribute__((address_space(4))) BatchPass *;
    using ItemPtr = const __attribute__((address_space(4))) BatchItem *;
    PassPtr passes = (PassPtr)b.passes;
    ItemPtr items = (ItemPtr)b.items;
    for (uint32_t it = b.i0 + blockIdx.x; it < b.i1; it += gridDim.x) {
        const uint32_t pi = items[it].pass, t0 = items[it].t0, t1 = items[it].t1;
        const auto &P = passes[pi];
        typename TK::Readout ro{P.last ? b.partials + 2 * (P.part + t0) : nullptr, P.zpos};
        TK::template run_range<true>(P.t, lds_raw, t0, t1, 1, ro);
    }
}

template <typename R, int LOG_NT, int LOG_R>
void launch_batch_inst(const BatchArgs &b, int grid, hipStream_t st)
{
    constexpr size_t bytes = TileKernel<R, LOG_NT, LOG_R, false, false>::LDS_BYTES;
    // once per process (a thread-safe static initialisation); a failure
    // throws, and the next launch tries again
    static const bool ready = [] {
        const void *fn = reinterpret_cast<const void *>(&k_batch<R, LOG_NT, LOG_R>);
        check_no_static_lds(fn, "batch kernel");
        // launches above the default dynamic LDS limit need the attribute first
        if (bytes > 65536) {
            hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
            if (e != hipSuccess)
                fail(QS_ERR_HIP, std::string("batch kernel attribute: ") + hipGetErrorString(e));
        }
        return true;
    }();
    (void)ready;
    hipLaunchKernelGGL((k_batch<R, LOG_NT, LOG_R>), dim3(grid), dim3(1 << LOG_NT), bytes, st, b);
    check_launch("batch launch");
}

// tile shapes of the batching form: 64 to 256 threads, 4..16 amplitudes each
template <typename R>
void launch_batch_t(const BatchArgs &b, int log_r, int log_nt, int grid, hipStream_t st)
{
#define QS_BATCH_CASE(NTB, RB)                          \
    if (log_nt == NTB && log_r == RB) {                 \
        launch_batch_inst<R, NTB, RB>(b, grid, st);     \
        return;                                         \
    }
    QS_BATCH_CASE(6, 2)
    QS_BATCH_CASE(6, 3)
    QS_BATCH_CASE(6, 4)
    QS_BATCH_CASE(7, 2)
    QS_BATCH_CASE(7, 3)
    QS_BATCH_CASE(7, 4)
    QS_BATCH_CASE(8, 3)
    QS_BATCH_CASE(8, 4)
#undef QS_BATCH_CASE
    fail(QS_ERR_UNSUPPORTED, "batch tile shape not instantiated (log_nt=" + std::to_string(log_nt) +
                                 ", log_r=" + std::to_string(log_r) + ")");
}

}  // namespace qsim
