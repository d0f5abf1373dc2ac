// Read-out kernels (paper, Section 2: measurement): norm, <Z_q> for every
// qubit in one read of the state, amplitude gather and the overlap of two
// states.  All sums are accumulated in FP64 and reduced in a fixed order
// (block partials, then one pass over the partials), so results do not depend
// on scheduling.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.cuh"
#include "kernels.h"

namespace qsim {

namespace {

constexpr int ZT = 256;          // threads per block
constexpr int ZT_BITS = 8;
constexpr int ZCHUNK_BITS = 18;  // largest chunk: 2^18 amplitudes per block

// Amplitudes per block = 2^L: at least 2^14, and at most 2^16 blocks.
inline int zchunk_bits(int n)
{
    int L = n - 16 > 14 ? n - 16 : 14;
    L = L < ZCHUNK_BITS ? L : ZCHUNK_BITS;
    return n < L ? n : L;
}

// Block b covers physical indices [b 2^L, (b+1) 2^L).  For each position p it
// writes S_p(block) = sum over its indices j with bit p set of |v_j|^2, and
// the block norm, into part[b * (n + 1) + ...].
template <typename R>
__global__ __launch_bounds__(ZT) void k_zsum(const Cplx<R> *__restrict__ s, int n, int L, double *part)
{
    __shared__ double tot[ZT];
    __shared__ double itb[ZCHUNK_BITS - ZT_BITS > 0 ? ZCHUNK_BITS - ZT_BITS : 1][ZT];
    const int tid = threadIdx.x;
    const int nthr = L >= ZT_BITS ? ZT : (1 << L);
    const int it_bits = L > ZT_BITS ? L - ZT_BITS : 0;
    const uint64_t base = (uint64_t)blockIdx.x << L;
    double total = 0.0;
    double acc[ZCHUNK_BITS - ZT_BITS > 0 ? ZCHUNK_BITS - ZT_BITS : 1];
#pragma unroll
    for (int b = 0; b < ZCHUNK_BITS - ZT_BITS; ++b)
        acc[b] = 0.0;
    if (tid < nthr) {
        const int iters = 1 << it_bits;
        for (int it = 0; it < iters; ++it) {
            const Cplx<R> a = s[base + ((uint64_t)it << ZT_BITS) + tid];
            const double re = (double)a.x, im = (double)a.y;
            const double p = re * re + im * im;
            total += p;
#pragma unroll
            for (int b = 0; b < ZCHUNK_BITS - ZT_BITS; ++b)
                if ((it >> b) & 1)
                    acc[b] += p;
        }
    }
    tot[tid] = tid < nthr ? total : 0.0;
#pragma unroll
    for (int b = 0; b < ZCHUNK_BITS - ZT_BITS; ++b)
        itb[b][tid] = acc[b];
    __syncthreads();
    // one thread per output, summing threads in index order
    const int outs = n + 1;
    for (int o = tid; o < outs; o += ZT) {
        double r = 0.0;
        if (o == 0) {
            for (int t = 0; t < nthr; ++t)
                r += tot[t];
        } else {
            const int p = o - 1;
            if (p < ZT_BITS && p < L) {
                for (int t = 0; t < nthr; ++t)
                    if ((t >> p) & 1)
                        r += tot[t];
            } else if (p < L) {
                for (int t = 0; t < nthr; ++t)
                    r += itb[p - ZT_BITS][t];
            } else if ((base >> p) & 1) {
                for (int t = 0; t < nthr; ++t)
                    r += tot[t];
            }
        }
        part[(uint64_t)blockIdx.x * outs + o] = r;
    }
}

// out[o] = sum over blocks of part[b][o]: thread t of block o sums the blocks
// b = t (mod 256) in order, then the 256 thread sums are added in a fixed tree.
__global__ __launch_bounds__(256) void k_sum_parts(const double *part, uint64_t nblocks, int outs, double *out)
{
    __shared__ double red[256];
    const int o = blockIdx.x;
    double r = 0.0;
    for (uint64_t b = threadIdx.x; b < nblocks; b += 256)
        r += part[b * outs + o];
    red[threadIdx.x] = r;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        out[o] = red[0];
}

// Fold the per-tile read-out of a tile pass into the sums of k_zsum (see
// ZFoldMap): output 0 is the sum over tiles of T, output 1 + p that of the
// probability of bit p.  Block (s, o) takes slice s of the tiles for output
// o: thread t of the block takes the slice's tiles t (mod 256) in order, the
// 256 sums are added in a fixed tree into work[s * outs + o], and
// k_sum_parts adds the slices in order.
static uint64_t zfold_slices(uint64_t tiles) { return std::min<uint64_t>(256, std::max<uint64_t>(1, tiles >> 10)); }

__global__ __launch_bounds__(256) void k_zfold(const double *parts, uint64_t tiles, uint64_t chunk, ZFoldMap m,
                                               int outs, double *work)
{
    __shared__ double red[256];
    const uint64_t s = blockIdx.x;
    const int o = blockIdx.y;
    const int v = o == 0 ? 0 : m.v[o - 1];
    const uint64_t rm = o == 0 ? 0 : m.rm[o - 1];
    const uint64_t t_end = std::min(tiles, (s + 1) * chunk);
    double r = 0.0;
    for (uint64_t t = s * chunk + threadIdx.x; t < t_end; t += 256) {
        const double T = parts[t];
        const bool odd = (__popcll(t & rm) & 1) != 0;
        if (o == 0)
            r += T;
        else if (v >= 1)
            r += odd ? T - parts[(uint64_t)v * tiles + t] : parts[(uint64_t)v * tiles + t];
        else if (odd)
            r += T;
    }
    red[threadIdx.x] = r;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        work[s * outs + o] = red[0];
}

template <typename R>
__global__ __launch_bounds__(256) void k_gather(const Cplx<R> *__restrict__ s, const uint64_t *idx, int64_t count,
                                                double *out)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) {
        const Cplx<R> a = s[idx[i]];
        out[2 * i] = (double)a.x;
        out[2 * i + 1] = (double)a.y;
    }
}

struct IndexMap {
    int n;
    uint8_t to[48];
    int identity;
};

constexpr int FT = 256;
constexpr int FCHUNK = 1 << 14;

// partials per block: [re <a|b>, im <a|b>, <a|a>, <b|b>, max |a - b|]
template <typename Ra, typename Rb>
__global__ __launch_bounds__(FT) void k_fid(const Cplx<Ra> *__restrict__ a, const Cplx<Rb> *__restrict__ b, uint64_t N,
                                            IndexMap map, double *part)
{
    __shared__ double red[5][FT];
    const uint64_t base = (uint64_t)blockIdx.x * FCHUNK;
    double sr = 0, si = 0, na = 0, nb = 0, mx = 0;
    for (int it = 0; it < FCHUNK / FT; ++it) {
        const uint64_t j = base + (uint64_t)it * FT + threadIdx.x;
        if (j >= N)
            break;
        uint64_t jb = j;
        if (!map.identity) {
            jb = 0;
#pragma unroll
            for (int p = 0; p < MAX_QUBITS; ++p)
                if (p < map.n)
                    jb |= ((j >> p) & 1ull) << map.to[p];
        }
        const Cplx<Ra> x = a[j];
        const Cplx<Rb> y = b[jb];
        const double xr = x.x, xi = x.y, yr = y.x, yi = y.y;
        sr += xr * yr + xi * yi;  // conj(x) * y
        si += xr * yi - xi * yr;
        na += xr * xr + xi * xi;
        nb += yr * yr + yi * yi;
        const double dr = xr - yr, di = xi - yi;
        const double d = sqrt(dr * dr + di * di);
        mx = d > mx ? d : mx;
    }
    red[0][threadIdx.x] = sr;
    red[1][threadIdx.x] = si;
    red[2][threadIdx.x] = na;
    red[3][threadIdx.x] = nb;
    red[4][threadIdx.x] = mx;
    __syncthreads();
    if (threadIdx.x < 5) {
        const int q = threadIdx.x;
        double r = 0;
        for (int t = 0; t < FT; ++t)
            r = q == 4 ? (red[q][t] > r ? red[q][t] : r) : r + red[q][t];
        part[(uint64_t)blockIdx.x * 5 + q] = r;
    }
}

// out[q] over the block partials: block q, thread t takes the blocks
// b = t (mod 256) in order, then a fixed tree over the 256 thread results
// (a sum for q < 4, a maximum for q = 4)
__global__ __launch_bounds__(256) void k_fid_final(const double *part, uint64_t nblocks, double *out)
{
    __shared__ double red[256];
    const int q = blockIdx.x;
    double r = 0;
    for (uint64_t b = threadIdx.x; b < nblocks; b += 256) {
        const double v = part[b * 5 + q];
        r = q == 4 ? (v > r ? v : r) : r + v;
    }
    red[threadIdx.x] = r;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const double x = red[threadIdx.x], y = red[threadIdx.x + w];
            red[threadIdx.x] = q == 4 ? (y > x ? y : x) : x + y;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        out[q] = red[0];
}

template <typename Ra, typename Rb>
void fid_t(const void *a, const void *b, int n, const IndexMap &m, double *work, double *out, hipStream_t st)
{
    const uint64_t N = 1ull << n;
    const uint64_t nb = (N + FCHUNK - 1) / FCHUNK;
    hipLaunchKernelGGL((k_fid<Ra, Rb>), dim3((unsigned)nb), dim3(FT), 0, st, reinterpret_cast<const Cplx<Ra> *>(a),
                       reinterpret_cast<const Cplx<Rb> *>(b), N, m, work);
    check_launch("fidelity");
    hipLaunchKernelGGL(k_fid_final, dim3(5), dim3(256), 0, st, work, nb, out);
    check_launch("fidelity final");
}

}  // namespace

size_t zsum_work_doubles(int n)
{
    const int L = zchunk_bits(n);
    return ((1ull << n) >> L) * (size_t)(n + 1);
}

void launch_zsum(const void *state, qs_dtype dt, int n, double *work, double *out, hipStream_t st)
{
    const int L = zchunk_bits(n);
    const uint64_t nb = (1ull << n) >> L;
    if (dt == QS_C64)
        hipLaunchKernelGGL(k_zsum<float>, dim3((unsigned)nb), dim3(ZT), 0, st,
                           reinterpret_cast<const Cplx<float> *>(state), n, L, work);
    else
        hipLaunchKernelGGL(k_zsum<double>, dim3((unsigned)nb), dim3(ZT), 0, st,
                           reinterpret_cast<const Cplx<double> *>(state), n, L, work);
    check_launch("zsum");
    hipLaunchKernelGGL(k_sum_parts, dim3(n + 1), dim3(256), 0, st, work, nb, n + 1, out);
    check_launch("zsum final");
}

size_t zfold_work_doubles(uint64_t tiles, int n) { return (size_t)zfold_slices(tiles) * (size_t)(n + 1); }

void launch_zfold(const double *parts, uint64_t tiles, int nv, int n, const ZFoldMap &m, double *work_dev,
                  double *out_dev, hipStream_t st)
{
    (void)nv;
    const uint64_t S = zfold_slices(tiles), chunk = (tiles + S - 1) / S;
    hipLaunchKernelGGL(k_zfold, dim3((unsigned)S, (unsigned)(n + 1)), dim3(256), 0, st, parts, tiles, chunk, m, n + 1,
                       work_dev);
    check_launch("zfold");
    hipLaunchKernelGGL(k_sum_parts, dim3(n + 1), dim3(256), 0, st, work_dev, S, n + 1, out_dev);
    check_launch("zfold final");
}

void launch_gather(const void *state, qs_dtype dt, const uint64_t *idx, int64_t count, double *out, hipStream_t st)
{
    if (count <= 0)
        return;
    const unsigned nb = (unsigned)((count + 255) / 256);
    if (dt == QS_C64)
        hipLaunchKernelGGL(k_gather<float>, dim3(nb), dim3(256), 0, st, reinterpret_cast<const Cplx<float> *>(state),
                           idx, count, out);
    else
        hipLaunchKernelGGL(k_gather<double>, dim3(nb), dim3(256), 0, st,
                           reinterpret_cast<const Cplx<double> *>(state), idx, count, out);
    check_launch("gather");
}

size_t fid_work_doubles(int n)
{
    const uint64_t N = 1ull << n;
    return (size_t)((N + FCHUNK - 1) / FCHUNK) * 5;
}

void launch_fidelity(const void *a, qs_dtype da, const void *b, qs_dtype db, int n, const std::vector<int> &map_b,
                     double *work, double *out, hipStream_t st)
{
    IndexMap m{};
    m.n = n;
    m.identity = 1;
    for (int p = 0; p < n; ++p) {
        m.to[p] = (uint8_t)map_b[p];
        if (map_b[p] != p)
            m.identity = 0;
    }
    if (da == QS_C64 && db == QS_C64)
        fid_t<float, float>(a, b, n, m, work, out, st);
    else if (da == QS_C64 && db == QS_C128)
        fid_t<float, double>(a, b, n, m, work, out, st);
    else if (da == QS_C128 && db == QS_C64)
        fid_t<double, float>(a, b, n, m, work, out, st);
    else
        fid_t<double, double>(a, b, n, m, work, out, st);
}

}  // namespace qsim
