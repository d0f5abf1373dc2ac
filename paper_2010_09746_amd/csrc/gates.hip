// Plain-form kernels: one launch per gate (paper, Section 2: gates update
// amplitudes in pairs), the in-place data movement of PermuteQubits and state
// preparation.
//
// Every kernel is bound by HBM traffic.  Threads take consecutive pair indices,
// so for a target position t >= log2(64) a wavefront reads two contiguous
// 64-amplitude runs; for lower t the pairs interleave inside the same cache
// lines and both halves of each line are consumed by the same wavefront.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.cuh"
#include "kernels.h"

namespace qsim {

namespace {

// Amplitude access: non-temporal when every 128-byte line a launch touches is
// read or written whole by one instruction (no qubit below the line size is
// split across instructions), cached otherwise, where the two halves of a line
// arrive from different instructions and the cache merges them.
template <bool NTA, typename C> __device__ __forceinline__ C ld(const C *p)
{
    if constexpr (NTA)
        return ld_stream(p);
    else
        return *p;
}
template <bool NTA, typename C> __device__ __forceinline__ void st(C *p, const C &v)
{
    if constexpr (NTA)
        st_stream(p, v);
    else
        *p = v;
}


constexpr int NT = 256;   // threads per block
constexpr int UNR = 4;    // pairs per thread, loads issued before use

__device__ __forceinline__ uint64_t insert_zero(uint64_t x, int b)
{
    const uint64_t lo = x & ((1ull << b) - 1);
    return ((x >> b) << (b + 1)) | lo;
}

template <typename R>
__global__ __launch_bounds__(NT) void k_set_basis(typename Cx<R>::T *s, uint64_t N, uint64_t x)
{
    using C = typename Cx<R>::T;
    // grid-stride over chunks of NT * UNR items (a launch is capped below 2^31 threads)
    for (uint64_t chunk = (uint64_t)blockIdx.x * NT * UNR; chunk < N; chunk += (uint64_t)gridDim.x * NT * UNR) {
        const uint64_t i0 = chunk + threadIdx.x;
    #pragma unroll
        for (int u = 0; u < UNR; ++u) {
            uint64_t i = i0 + (uint64_t)u * NT;
            if (i < N) {
                C v;
                v.x = i == x ? R(1) : R(0);
                v.y = R(0);
                st_stream(&s[i], v);
            }
        }
    }
}

// (a_i, a_j) <- U (a_i, a_j) for j = i | 2^t, optionally only where bit c = 1.
template <typename R, bool CTRL, bool NTA>
__global__ __launch_bounds__(NT) void k_pair_u(typename Cx<R>::T *__restrict__ s, uint64_t npairs,
                                               int t, int c_lo, int c_hi, uint64_t cbit, Mat<R> m)
{
    using C = typename Cx<R>::T;
    // grid-stride over chunks of NT * UNR items (a launch is capped below 2^31 threads)
    for (uint64_t chunk = (uint64_t)blockIdx.x * NT * UNR; chunk < npairs; chunk += (uint64_t)gridDim.x * NT * UNR) {
        const uint64_t p0 = chunk + threadIdx.x;
        C a[UNR], b[UNR];
        uint64_t ii[UNR];
    #pragma unroll
        for (int u = 0; u < UNR; ++u) {
            uint64_t p = p0 + (uint64_t)u * NT;
            uint64_t i;
            if (CTRL)
                i = insert_zero(insert_zero(p, c_lo), c_hi) | cbit;
            else
                i = insert_zero(p, t);
            ii[u] = i;
            if (p < npairs) {
                a[u] = ld<NTA>(&s[i]);
                b[u] = ld<NTA>(&s[i | (1ull << t)]);
            }
        }
    #pragma unroll
        for (int u = 0; u < UNR; ++u) {
            uint64_t p = p0 + (uint64_t)u * NT;
            if (p < npairs) {
                C x = a[u], y = b[u];
                st<NTA>(&s[ii[u]], m.row0(x, y));
                st<NTA>(&s[ii[u] | (1ull << t)], m.row1(x, y));
            }
        }
    }
}

// controlled X: exchange a_i and a_j where bit c = 1
template <typename R, bool NTA>
__global__ __launch_bounds__(NT) void k_cx(typename Cx<R>::T *__restrict__ s, uint64_t nquads, int t,
                                           int lo, int hi, uint64_t cbit)
{
    using C = typename Cx<R>::T;
    // grid-stride over chunks of NT * UNR items (a launch is capped below 2^31 threads)
    for (uint64_t chunk = (uint64_t)blockIdx.x * NT * UNR; chunk < nquads; chunk += (uint64_t)gridDim.x * NT * UNR) {
        const uint64_t p0 = chunk + threadIdx.x;
        C a[UNR], b[UNR];
        uint64_t ii[UNR];
    #pragma unroll
        for (int u = 0; u < UNR; ++u) {
            uint64_t p = p0 + (uint64_t)u * NT;
            ii[u] = insert_zero(insert_zero(p, lo), hi) | cbit;
            if (p < nquads) {
                a[u] = ld<NTA>(&s[ii[u]]);
                b[u] = ld<NTA>(&s[ii[u] | (1ull << t)]);
            }
        }
    #pragma unroll
        for (int u = 0; u < UNR; ++u) {
            uint64_t p = p0 + (uint64_t)u * NT;
            if (p < nquads) {
                st<NTA>(&s[ii[u]], b[u]);
                st<NTA>(&s[ii[u] | (1ull << t)], a[u]);
            }
        }
    }
}

// controlled Z: negate a_i where both bits are 1
template <typename R, bool NTA>
__global__ __launch_bounds__(NT) void k_cz(typename Cx<R>::T *__restrict__ s, uint64_t nquads, int lo,
                                           int hi, uint64_t both)
{
    using C = typename Cx<R>::T;
    // grid-stride over chunks of NT * UNR items (a launch is capped below 2^31 threads)
    for (uint64_t chunk = (uint64_t)blockIdx.x * NT * UNR; chunk < nquads; chunk += (uint64_t)gridDim.x * NT * UNR) {
        const uint64_t p0 = chunk + threadIdx.x;
        C a[UNR];
        uint64_t ii[UNR];
    #pragma unroll
        for (int u = 0; u < UNR; ++u) {
            uint64_t p = p0 + (uint64_t)u * NT;
            ii[u] = insert_zero(insert_zero(p, lo), hi) | both;
            if (p < nquads)
                a[u] = ld<NTA>(&s[ii[u]]);
        }
    #pragma unroll
        for (int u = 0; u < UNR; ++u) {
            uint64_t p = p0 + (uint64_t)u * NT;
            if (p < nquads) {
                C v = a[u];
                v.x = -v.x;
                v.y = -v.y;
                st<NTA>(&s[ii[u]], v);
            }
        }
    }
}

// In-place exchange of chunks of 2^c0 amplitudes: chunk x0 and chunk J(x0),
// where J moves bit p of the index to bit pi[p] (an involution, identity on
// positions below c0).  The pair is exchanged by the chunk with x0 < J(x0).
struct Involution {
    int n_moved;
    uint8_t from[48], to[48];
    uint64_t moved_mask;
};

template <typename R, bool NTA>
__global__ __launch_bounds__(NT) void k_involution(typename Cx<R>::T *__restrict__ s, uint64_t N, int c0,
                                                   Involution J)
{
    using C = typename Cx<R>::T;
    // grid-stride over chunks of NT * UNR items (a launch is capped below 2^31 threads)
    for (uint64_t chunk = (uint64_t)blockIdx.x * NT * UNR; chunk < N; chunk += (uint64_t)gridDim.x * NT * UNR) {
        const uint64_t i0 = chunk + threadIdx.x;
    #pragma unroll
        for (int u = 0; u < UNR; ++u) {
            uint64_t x = i0 + (uint64_t)u * NT;
            if (x >= N)
                continue;
            uint64_t y = x & ~J.moved_mask;
    #pragma unroll
            for (int k = 0; k < MAX_QUBITS; ++k)
                if (k < J.n_moved)
                    y |= ((x >> J.from[k]) & 1ull) << J.to[k];
            if (x < y) {
                const C a = ld<NTA>(&s[x]), b = ld<NTA>(&s[y]);
                st<NTA>(&s[x], b);
                st<NTA>(&s[y], a);
            }
        }
        (void)c0;
    }
}

// blocks for items, at most 2^31 threads per launch (the kernels stride over
// the rest)
inline unsigned blocks_for(uint64_t items)
{
    uint64_t b = (items + (uint64_t)NT * UNR - 1) / ((uint64_t)NT * UNR);
    b = std::min<uint64_t>(b, (1ull << 31) / NT);
    return (unsigned)(b ? b : 1);
}

// qubits below this index split a 128-byte line
template <typename R> constexpr int line_bits() { return sizeof(typename Cx<R>::T) == 16 ? 3 : 4; }

template <typename R, bool NTA>
void plain_gate_nt(typename Cx<R>::T *s, int n, const qs_gate &g, hipStream_t st)
{
    switch (g.kind) {
    case QS_GATE_U: {
        uint64_t np = 1ull << (n - 1);
        hipLaunchKernelGGL((k_pair_u<R, false, NTA>), dim3(blocks_for(np)), dim3(NT), 0, st, s, np, g.q0, 0, 0,
                           0ull, Mat<R>(g.u));
        break;
    }
    case QS_GATE_CU: {
        uint64_t nq = 1ull << (n - 2);
        int lo = g.q0 < g.q1 ? g.q0 : g.q1, hi = g.q0 < g.q1 ? g.q1 : g.q0;
        hipLaunchKernelGGL((k_pair_u<R, true, NTA>), dim3(blocks_for(nq)), dim3(NT), 0, st, s, nq, g.q1, lo, hi,
                           1ull << g.q0, Mat<R>(g.u));
        break;
    }
    case QS_GATE_CX: {
        uint64_t nq = 1ull << (n - 2);
        int lo = g.q0 < g.q1 ? g.q0 : g.q1, hi = g.q0 < g.q1 ? g.q1 : g.q0;
        hipLaunchKernelGGL((k_cx<R, NTA>), dim3(blocks_for(nq)), dim3(NT), 0, st, s, nq, g.q1, lo, hi,
                           1ull << g.q0);
        break;
    }
    case QS_GATE_CZ: {
        uint64_t nq = 1ull << (n - 2);
        int lo = g.q0 < g.q1 ? g.q0 : g.q1, hi = g.q0 < g.q1 ? g.q1 : g.q0;
        hipLaunchKernelGGL((k_cz<R, NTA>), dim3(blocks_for(nq)), dim3(NT), 0, st, s, nq, lo, hi,
                           (1ull << g.q0) | (1ull << g.q1));
        break;
    }
    default:
        fail(QS_ERR_ARG, "unknown gate kind");
    }
    check_launch("plain gate");
}

template <typename R>
void plain_gate_t(void *state, int n, const qs_gate &g, hipStream_t st)
{
    using C = typename Cx<R>::T;
    C *s = reinterpret_cast<C *>(state);
    // the lowest qubit the launch splits on: the target, or the lower of two
    const int low = g.kind == QS_GATE_U ? g.q0 : (g.q0 < g.q1 ? g.q0 : g.q1);
    if (low >= line_bits<R>())
        plain_gate_nt<R, true>(s, n, g, st);
    else
        plain_gate_nt<R, false>(s, n, g, st);
}

}  // namespace

void launch_set_basis(void *state, qs_dtype dt, int n, uint64_t x, hipStream_t st)
{
    uint64_t N = 1ull << n;
    if (dt == QS_C64)
        hipLaunchKernelGGL(k_set_basis<float>, dim3(blocks_for(N)), dim3(NT), 0, st,
                           reinterpret_cast<Cplx<float> *>(state), N, x);
    else
        hipLaunchKernelGGL(k_set_basis<double>, dim3(blocks_for(N)), dim3(NT), 0, st,
                           reinterpret_cast<Cplx<double> *>(state), N, x);
    check_launch("set_basis");
}

void launch_plain_gate(void *state, qs_dtype dt, int n, const qs_gate &g, hipStream_t st)
{
    if (g.kind != QS_GATE_U && n < 2)
        fail(QS_ERR_ARG, "two-qubit gate on a one-qubit state");
    if (dt == QS_C64)
        plain_gate_t<float>(state, n, g, st);
    else
        plain_gate_t<double>(state, n, g, st);
}

void launch_involution(void *state, qs_dtype dt, int n, const std::vector<int> &pi, hipStream_t st)
{
    Involution J{};
    int c0 = n;
    for (int p = 0; p < n; ++p) {
        if (pi[p] != p) {
            if (pi[pi[p]] != p)
                fail(QS_ERR_ARG, "internal: position map is not an involution");
            J.from[J.n_moved] = (uint8_t)p;
            J.to[J.n_moved] = (uint8_t)pi[p];
            J.moved_mask |= 1ull << p;
            ++J.n_moved;
            c0 = p < c0 ? p : c0;
        }
    }
    if (J.n_moved == 0)
        return;
    uint64_t N = 1ull << n;
    // a pair is whole lines apart only when no moved position is below the line
    if (dt == QS_C64) {
        auto *s = reinterpret_cast<Cplx<float> *>(state);
        if (c0 >= line_bits<float>())
            hipLaunchKernelGGL((k_involution<float, true>), dim3(blocks_for(N)), dim3(NT), 0, st, s, N, c0, J);
        else
            hipLaunchKernelGGL((k_involution<float, false>), dim3(blocks_for(N)), dim3(NT), 0, st, s, N, c0, J);
    } else {
        auto *s = reinterpret_cast<Cplx<double> *>(state);
        if (c0 >= line_bits<double>())
            hipLaunchKernelGGL((k_involution<double, true>), dim3(blocks_for(N)), dim3(NT), 0, st, s, N, c0, J);
        else
            hipLaunchKernelGGL((k_involution<double, false>), dim3(blocks_for(N)), dim3(NT), 0, st, s, N, c0, J);
    }
    check_launch("involution");
}

}  // namespace qsim
