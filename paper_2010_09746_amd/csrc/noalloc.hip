// qs_run_program_noalloc: qs_run_program for callers that cannot allocate
// device memory.  The only device memory qs_run_program adds to the state and
// the program is the program's operation table (the records the fused tile
// passes read); here it is staged in a fixed array in the library's own device
// memory instead of a buffer allocated on first run.
//
// Each device that loads the library holds one copy of the array, at its own
// address: the host looks that address up once per device, with the device
// current, and only ever passes the looked-up pointer to kernels and copies.
// Every call on a device overwrites the array with its own table; calls that
// overlap on one device (other streams, other threads) race for it.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "internal.h"

using namespace qsim;

namespace {

constexpr size_t NOALLOC_MAX_OPS = QS_NOALLOC_MAX_OPS;
constexpr int MAX_DEVICES = 64;

}  // namespace

// the operation table of the running call (3.25 MiB per device)
static __device__ __align__(256) unsigned char scratch[NOALLOC_MAX_OPS * sizeof(TileOp)];

namespace {

std::mutex g_mu;
void *g_scratch[MAX_DEVICES] = {};

// Device address of this device's copy of the array, looked up on the first
// call on the device (the device is current: the caller checked it).
void *scratch_on(int dev)
{
    if (dev < 0 || dev >= MAX_DEVICES)
        fail(QS_ERR_UNSUPPORTED, "device index beyond the allocation-free entry point's table");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || ptr == nullptr) {
            (void)hipGetLastError();
            fail(QS_ERR_HIP, std::string("hipGetSymbolAddress(operation scratch): ") + hipGetErrorString(e));
        }
        g_scratch[dev] = ptr;
    }
    return g_scratch[dev];
}

}  // namespace

extern "C" qs_status qs_run_program_noalloc(qs_state *s, const qs_program *p)
{
    return guarded([&] {
        if (s == nullptr || p == nullptr)
            fail(QS_ERR_ARG, "NULL argument");
        const Program &P = p->p;
        check_program_on(s, P);
        if (P.ops.size() > NOALLOC_MAX_OPS)
            fail(QS_ERR_ARG, "program has " + std::to_string(P.ops.size()) +
                                 " tile operations; the allocation-free entry point holds at most " +
                                 std::to_string(NOALLOC_MAX_OPS));
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess || cur != state_device(s))
            fail(QS_ERR_STATE, "the state's device must be the current device");
        void *ops = scratch_on(cur);
        const hipStream_t st = reinterpret_cast<hipStream_t>(state_stream(s));
        if (!P.ops.empty()) {
            // ordered on the state's stream after the work already there,
            // which may include an earlier call's passes reading the array
            const hipError_t e =
                hipMemcpyAsync(ops, P.ops.data(), P.ops.size() * sizeof(TileOp), hipMemcpyHostToDevice, st);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                fail(QS_ERR_HIP, std::string("hipMemcpyAsync(operation scratch): ") + hipGetErrorString(e));
            }
        }
        run_program_with_ops(s, P, reinterpret_cast<const TileOp *>(ops));
    });
}
