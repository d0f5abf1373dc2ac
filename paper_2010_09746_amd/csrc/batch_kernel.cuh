// Batching form: many independent circuits of different sizes, advanced one
// pass level at a time.  A level holds every circuit's tile pass of that index;
// its work items (ranges of tiles) are independent, so one persistent launch
// per level strides over them with no waiting between workgroups, and the
// ordering between a circuit's consecutive passes comes from the launch order.
// The whole sequence of level launches is captured once in a HIP graph.
#pragma once

#include "kernels.h"
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

// ---------------------------------------------------------------------------
// Single-launch executor of a batch.  One persistent launch takes work items
// (ranges of tiles of one pass) in ticket order; an item whose circuit's
// previous pass has not completed waits for it.  The item list is ordered so
// that every dependency precedes its dependents, and a workgroup takes a
// ticket only while it runs, so the lowest unfinished ticket always belongs to
// a running workgroup whose dependency is complete: the launch drains.
//
// Memory ordering across the device (its L2 caches are per XCD and not
// coherent with each other for ordinary device memory): a finished item's
// stores are complete (every wavefront waits for its stores) before the
// workgroup's barrier; one thread then releases at agent scope (writes back
// the L2) and adds its tile count to the pass's counter.  A waiter polls the
// counter with agent-scope atomic loads and acquires at agent scope
// (invalidates its caches) before the barrier that lets its workgroup read
// the state.  A wait gives up after a bounded time, or as soon as the host
// sets the abort flag or another wait has given up; the launch then ends
// early with the error flag set, and the host reports it.
template <typename R> struct QueueKernel {
    // one component per re-layout round (LDS holds half a tile): moving
    // whole amplitudes made the kernel need more registers (complex64: 129
    // VGPRs, 3 wavefronts per SIMD, instead of 111)
    static constexpr bool HALF = true;
    template <int SH> using TK = TileKernel<R, QUEUE_LOG_NT, SH, HALF, false>;
    static constexpr uint32_t mx(uint32_t a, uint32_t b) { return a > b ? a : b; }
    static constexpr uint32_t TILE_LDS =
        mx(mx(TK<1>::LDS_BYTES, TK<2>::LDS_BYTES), mx(TK<3>::LDS_BYTES, TK<4>::LDS_BYTES));
    static constexpr uint32_t LDS_BYTES = TILE_LDS + 16;  // + the words one thread broadcasts
};

// Release and acquire at device scope, each followed by a wait for the
// cache operation it issues.  The compiler's own sequence for a release
// writes back the L2 (buffer_wbl2) and, when no store of the wavefront is
// outstanding, issues the following atomic without waiting for that
// write-back: the counter could then be seen on another XCD before the data
// it publishes has reached memory.
__device__ __forceinline__ void release_device()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
}
__device__ __forceinline__ void acquire_device()
{
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
}

// Wait until pass `dep` has completed `need` tiles (thread 0 only).  Returns
// 0 when it has, 1 when the wait gave up.
__device__ __forceinline__ uint32_t queue_wait(const QueueArgs &q, int dep, uint32_t need)
{
    if (q.wait_ticks == 0) {
        // every wait gives up at once (the host's test of the give-up path)
        __hip_atomic_store(&q.flags[1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        return 1;
    }
    if (__hip_atomic_load(&q.done[dep], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
        const uint64_t start = __builtin_amdgcn_s_memrealtime();
        for (uint32_t i = 1;; ++i) {
            __builtin_amdgcn_s_sleep(2);
            if (__hip_atomic_load(&q.done[dep], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need)
                break;
            if ((i & 63u) == 0) {
                if (__hip_atomic_load(&q.flags[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0u ||
                    __hip_atomic_load(&q.flags[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0u)
                    return 1;
                if (__builtin_amdgcn_s_memrealtime() - start > q.wait_ticks) {
                    __hip_atomic_store(&q.flags[1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    return 1;
                }
            }
        }
    }
    acquire_device();
    return 0;
}

template <typename R>
__global__ __launch_bounds__(256) void k_batch_queue(QueueArgs q)
{
    using QK = QueueKernel<R>;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    uint32_t *bc = reinterpret_cast<uint32_t *>(lds_raw + QK::TILE_LDS);
    using PassPtr = const __attribute__((address_space(4))) BatchPass *;
    using ItemPtr = const __attribute__((address_space(4))) QueueItem *;
    PassPtr passes = (PassPtr)q.passes;
    ItemPtr items = (ItemPtr)q.items;
    const uint32_t tid = threadIdx.x;
    for (;;) {
        if (tid == 0) {
            const uint32_t t = __hip_atomic_fetch_add(q.next, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            uint32_t stop = t >= q.n_items ? 1u : 0u;
            if (!stop && items[t].dep >= 0)
                stop = queue_wait(q, items[t].dep, items[t].need);
            bc[0] = t;
            bc[1] = stop;
        }
        __syncthreads();
        const uint32_t t = bc[0], stop = bc[1];
        __syncthreads();  // every thread has read the words before they change
        if (stop)
            break;
        const uint32_t pi = items[t].pass, t0 = items[t].t0, t1 = items[t].t1, sh = items[t].shape;
        const auto &P = passes[pi];
        double *part = P.last ? q.partials + 2 * (P.part + t0) : nullptr;
        switch (sh) {
        case 1: QK::template TK<1>::template run_range<false, true>(P.t, lds_raw, t0, t1, 1, {part, P.zpos}); break;
        case 2: QK::template TK<2>::template run_range<false, true>(P.t, lds_raw, t0, t1, 1, {part, P.zpos}); break;
        case 3: QK::template TK<3>::template run_range<false, true>(P.t, lds_raw, t0, t1, 1, {part, P.zpos}); break;
        default: QK::template TK<4>::template run_range<false, true>(P.t, lds_raw, t0, t1, 1, {part, P.zpos}); break;
        }
        // every wavefront's stores (and read-out partials) have completed
        __builtin_amdgcn_s_waitcnt(0x0F70);
        __syncthreads();
        if (tid == 0) {
            release_device();
            const uint32_t cnt = t1 - t0;
            const uint32_t before = __hip_atomic_fetch_add(&q.done[pi], cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // the workgroup that completes a circuit's last pass reduces its
            // read-out partials
            bc[2] = (P.last && before + cnt == P.ntiles) ? 1u : 0u;
            if (bc[2])
                acquire_device();
        }
        __syncthreads();
        if (bc[2]) {
            const int c = P.circuit;
            const double *pp = q.partials + 2 * q.part_off[c];
            const uint32_t cnt = q.part_cnt[c];
            double nrm = 0.0, z = 0.0;
            for (uint32_t i = tid; i < cnt; i += 256) {
                nrm += pp[2 * i];
                z += pp[2 * i + 1];
            }
            double *red = reinterpret_cast<double *>(lds_raw);
            red[tid] = nrm;
            red[256 + tid] = z;
            __syncthreads();
            for (uint32_t w = 128; w > 0; w >>= 1) {
                if (tid < w) {
                    red[tid] += red[tid + w];
                    red[256 + tid] += red[256 + tid + w];
                }
                __syncthreads();
            }
            if (tid == 0) {
                q.out[2 * c] = red[256];
                q.out[2 * c + 1] = red[0];
            }
        }
        __syncthreads();  // LDS and the broadcast words are reused by the next item
    }
}

template <typename R> void launch_batch_queue_t(const QueueArgs &q, int grid, hipStream_t st)
{
    constexpr size_t bytes = QueueKernel<R>::LDS_BYTES;
    const void *fn = reinterpret_cast<const void *>(&k_batch_queue<R>);
    static const bool ready = [fn] {
        check_no_static_lds(fn, "batch queue kernel");
        if (bytes > 65536) {
            hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
            if (e != hipSuccess)
                fail(QS_ERR_HIP, std::string("batch queue kernel attribute: ") + hipGetErrorString(e));
        }
        return true;
    }();
    (void)ready;
    hipLaunchKernelGGL((k_batch_queue<R>), dim3(grid), dim3(256), bytes, st, q);
    check_launch("batch queue launch");
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
