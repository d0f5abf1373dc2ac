// Fused tile pass: one workgroup loads a tile of 2^K amplitudes, applies a run
// of gates that act on the tile's qubits, and stores the tile back in place.
//
// The tile is the set of amplitudes whose physical index has fixed bits
// outside K chosen positions pos[0..K) (the local qubits of the permutation
// pass, paper, Section 3).  With pos = 0..K-1 the tile is a contiguous block;
// when the pass only relabels qubits the tile gathers strided runs.
//
// Data path per tile:
//   HBM -> LDS        coalesced: tile-local index t = j*NT + tid
//   LDS -> registers  layout chosen per group of gates (OP_REMAP): the
//                     register slots of a thread hold the 2^LOG_R amplitudes
//                     whose tile-local indices differ in the LOG_R "register
//                     bits"; the remaining bits come from the thread id
//   gates             one-qubit updates and exchanges on register bits run
//                     inside a thread; diagonal gates and controls on any bit
//                     (or on a position outside the tile) are evaluated from
//                     the tile-local index and the tile's base index
//   registers -> LDS -> HBM  coalesced store
#pragma once

#include <hip/hip_runtime.h>

#include "common.cuh"

namespace qsim {

template <typename R, int LOG_NT, int LOG_R> struct TileKernel {
    using C = typename Cx<R>::T;
    static constexpr int NT = 1 << LOG_NT, NR = 1 << LOG_R, K = LOG_NT + LOG_R;

    // register slot pair (j, j | 2^S) for pair index jj
    template <int S> static constexpr int pair_lo(int jj)
    {
        return ((jj >> S) << (S + 1)) | (jj & ((1 << S) - 1));
    }

    // dense 2x2 on slot S, in place; with CTRL only where the tile-local index
    // matches: (idx & cm) == cv
    template <int S, bool CTRL>
    static __device__ __forceinline__ void bfly(C (&v)[NR], const Mat<R> &m, uint32_t cm, uint32_t cv, uint32_t tbase,
                                                const uint32_t (&offs)[NR])
    {
#pragma unroll
        for (int jj = 0; jj < NR / 2; ++jj) {
            const int j = pair_lo<S>(jj), j1 = j | (1 << S);
            if (CTRL) {
                C x = v[j], y = v[j1];
                m.apply(x, y);
                const bool p = ((tbase | offs[j]) & cm) == cv;
                v[j].x = p ? x.x : v[j].x;
                v[j].y = p ? x.y : v[j].y;
                v[j1].x = p ? y.x : v[j1].x;
                v[j1].y = p ? y.y : v[j1].y;
            } else {
                m.apply(v[j], v[j1]);
            }
        }
    }

    template <int S>
    static __device__ __forceinline__ void xswap(C (&v)[NR], uint32_t cm, uint32_t cv, uint32_t tbase,
                                                 const uint32_t (&offs)[NR])
    {
#pragma unroll
        for (int jj = 0; jj < NR / 2; ++jj) {
            const int j = pair_lo<S>(jj), j1 = j | (1 << S);
            const C x = v[j], y = v[j1];
            const bool p = ((tbase | offs[j]) & cm) == cv;
            v[j].x = p ? y.x : x.x;
            v[j].y = p ? y.y : x.y;
            v[j1].x = p ? x.x : y.x;
            v[j1].y = p ? x.y : y.y;
        }
    }

    template <int S = 0>
    static __device__ __forceinline__ void dispatch_u(int slot, C (&v)[NR], const Mat<R> &m, uint32_t cm, uint32_t cv,
                                                      uint32_t tbase, const uint32_t (&offs)[NR])
    {
        if constexpr (S < LOG_R) {
            if (slot == S) {
                if (cm == 0)
                    bfly<S, false>(v, m, cm, cv, tbase, offs);
                else
                    bfly<S, true>(v, m, cm, cv, tbase, offs);
            } else {
                dispatch_u<S + 1>(slot, v, m, cm, cv, tbase, offs);
            }
        }
    }

    template <int S = 0>
    static __device__ __forceinline__ void dispatch_x(int slot, C (&v)[NR], uint32_t cm, uint32_t cv, uint32_t tbase,
                                                      const uint32_t (&offs)[NR])
    {
        if constexpr (S < LOG_R) {
            if (slot == S)
                xswap<S>(v, cm, cv, tbase, offs);
            else
                dispatch_x<S + 1>(slot, v, cm, cv, tbase, offs);
        }
    }

    template <typename P> static __device__ __forceinline__ uint32_t bitperm(uint32_t x, P perm)
    {
        uint32_t y = 0;
#pragma unroll
        for (int b = 0; b < K; ++b)
            y |= ((x >> b) & 1u) << perm[b];
        return y;
    }

    // deposit of the tile's register-slot bits j into the positions pos[LOG_NT..K)
    template <typename A> static __device__ __forceinline__ uint64_t slot_offset(const A &a, int j)
    {
        uint64_t dj = 0;
#pragma unroll
        for (int b = 0; b < LOG_R; ++b)
            if ((j >> b) & 1)
                dj |= 1ull << a.pos[LOG_NT + b];
        return dj;
    }

    using OpPtr = const __attribute__((address_space(4))) TileOp *;

    // the fields of one operation, held in scalar registers
    struct OpV {
        int32_t kind, slot;
        uint32_t cmask, regs;
        uint64_t hmask, hbit;
        double m[8];
    };

    static __device__ __forceinline__ OpV fetch(OpPtr ops, int i)
    {
        OpV o;
        o.kind = ops[i].kind;
        o.slot = ops[i].slot;
        o.cmask = ops[i].cmask;
        o.regs = ops[i].regs;
        o.hmask = ops[i].hmask;
        o.hbit = ops[i].hbit;
#pragma unroll
        for (int q = 0; q < 8; ++q)
            o.m[q] = ops[i].m[q];
        return o;
    }

    // Register slot j holds the amplitude of register pattern j ^ fl: an
    // exchange (X) whose control is the same for the whole tile flips a bit of
    // fl instead of moving data.  F is fl deposited into tile bits, so the
    // tile-local index of slot j is (tbase | offs[j]) ^ F.
    // Per-tile read-out of the final amplitudes: sum |a|^2 and sum |a|^2 (1 - 2 b)
    // where b is the bit at physical position zpos (the first qubit), reduced
    // over the workgroup in a fixed order and written to out[0..1].
    struct Readout {
        double *out;  // NULL: none
        int zpos;
    };

    // One tile.  A is TileArgs, read from kernel arguments or from device
    // memory; tile is the tile number (index over the positions outside it).
    template <typename A>
    static __device__ __forceinline__ void run(const A &a, unsigned char *lds_raw, uint64_t tile, Readout ro)
    {
        C *lds = reinterpret_cast<C *>(lds_raw);
        C *st = reinterpret_cast<C *>(a.state);
        OpPtr ops = (OpPtr)(a.ops);
        const uint32_t tid = threadIdx.x;

        // base index: the tile number with a zero inserted at every tile position
        // (positions ascending)
        uint64_t base = tile;
#pragma unroll
        for (int b = 0; b < K; ++b) {
            const int p = a.pos[b];
            base = ((base >> p) << (p + 1)) | (base & ((1ull << p) - 1));
        }
        uint64_t dtid = 0;
#pragma unroll
        for (int b = 0; b < LOG_NT; ++b)
            dtid |= (uint64_t)((tid >> b) & 1u) << a.pos[b];

        C v[NR];
#pragma unroll
        for (int j = 0; j < NR; ++j)
            v[j] = st[base + dtid + slot_offset(a, j)];
#pragma unroll
        for (int j = 0; j < NR; ++j)
            lds[j * NT + tid] = v[j];
        __syncthreads();

        uint32_t offs[NR];
#pragma unroll
        for (int j = 0; j < NR; ++j)
            offs[j] = 0;
        uint32_t tbase = 0, regs = 0, fl = 0, F = 0;
        bool have = false;

        const int n_ops = a.n_ops;
        for (int oi = 0; oi < n_ops; ++oi) {
            const OpV cur = fetch(ops, oi);
            const int kind = cur.kind;
            if (kind == OP_REMAP) {
                if (have) {
#pragma unroll
                    for (int j = 0; j < NR; ++j)
                        lds[(tbase | offs[j]) ^ F] = v[j];
                    __syncthreads();
                }
                regs = cur.regs;
                uint32_t regmask = 0;
                uint32_t rb[LOG_R];
#pragma unroll
                for (int s = 0; s < LOG_R; ++s) {
                    rb[s] = (regs >> (4 * s)) & 15u;
                    regmask |= 1u << rb[s];
                }
#pragma unroll
                for (int j = 0; j < NR; ++j) {
                    uint32_t o = 0;
#pragma unroll
                    for (int s = 0; s < LOG_R; ++s)
                        if ((j >> s) & 1)
                            o |= 1u << rb[s];
                    offs[j] = o;
                }
                tbase = 0;
                int tbit = 0;
#pragma unroll
                for (int b = 0; b < K; ++b) {
                    if (!((regmask >> b) & 1u)) {
                        tbase |= ((tid >> tbit) & 1u) << b;
                        ++tbit;
                    }
                }
#pragma unroll
                for (int j = 0; j < NR; ++j)
                    v[j] = lds[tbase | offs[j]];
                __syncthreads();
                fl = 0;
                F = 0;
                have = true;
            } else if ((base & cur.hmask) == cur.hmask) {
                const uint32_t cm = cur.cmask;
                const uint32_t cv = cm & ~F;  // (idx ^ F) & cm == cm  <=>  idx & cm == cm & ~F
                if (kind == OP_U) {
                    Mat<R> m;
                    const bool sw = (fl >> cur.slot) & 1u;
                    // with the slot's pattern bit flipped, rows and columns trade places
                    m.a[0] = (R)(sw ? cur.m[6] : cur.m[0]);
                    m.a[1] = (R)(sw ? cur.m[7] : cur.m[1]);
                    m.a[2] = (R)(sw ? cur.m[4] : cur.m[2]);
                    m.a[3] = (R)(sw ? cur.m[5] : cur.m[3]);
                    m.a[4] = (R)(sw ? cur.m[2] : cur.m[4]);
                    m.a[5] = (R)(sw ? cur.m[3] : cur.m[5]);
                    m.a[6] = (R)(sw ? cur.m[0] : cur.m[6]);
                    m.a[7] = (R)(sw ? cur.m[1] : cur.m[7]);
                    dispatch_u(cur.slot, v, m, cm, cv, tbase, offs);
                } else if (kind == OP_X) {
                    if (cm == 0) {
                        fl ^= 1u << cur.slot;
                        F ^= 1u << ((regs >> (4 * cur.slot)) & 15u);
                    } else {
                        dispatch_x(cur.slot, v, cm, cv, tbase, offs);
                    }
                } else if (kind == OP_NEG) {
#pragma unroll
                    for (int j = 0; j < NR; ++j) {
                        const bool p = ((tbase | offs[j]) & cm) == cv;
                        v[j].x = p ? -v[j].x : v[j].x;
                        v[j].y = p ? -v[j].y : v[j].y;
                    }
                } else {  // OP_DIAG
                    const R d0r = (R)cur.m[0], d0i = (R)cur.m[1], d1r = (R)cur.m[2], d1i = (R)cur.m[3];
                    const int tb = cur.slot;
                    const bool hsel = (base & cur.hbit) != 0;
#pragma unroll
                    for (int j = 0; j < NR; ++j) {
                        const uint32_t idx = (tbase | offs[j]) ^ F;
                        const bool p = (idx & cm) == cm;
                        const bool sel = tb >= 0 ? ((idx >> tb) & 1u) != 0 : hsel;
                        const R dr = sel ? d1r : d0r, di = sel ? d1i : d0i;
                        const C x = v[j];
                        const R nr = dr * x.x - di * x.y, ni = dr * x.y + di * x.x;
                        v[j].x = p ? nr : x.x;
                        v[j].y = p ? ni : x.y;
                    }
                }
            }
        }

        if (have) {
            if (a.has_perm) {
#pragma unroll
                for (int j = 0; j < NR; ++j)
                    lds[bitperm((tbase | offs[j]) ^ F, a.perm)] = v[j];
            } else {
#pragma unroll
                for (int j = 0; j < NR; ++j)
                    lds[(tbase | offs[j]) ^ F] = v[j];
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < NR; ++j)
                v[j] = lds[j * NT + tid];
        } else {
#pragma unroll
            for (int j = 0; j < NR; ++j) {
                const uint32_t t = (uint32_t)(j * NT) + tid;
                const uint32_t src = a.has_perm ? bitperm(t, a.pinv) : t;
                v[j] = lds[src];
            }
        }
#pragma unroll
        for (int j = 0; j < NR; ++j)
            st[base + dtid + slot_offset(a, j)] = v[j];
        if (ro.out)
            readout(a, v, base, dtid, ro, reinterpret_cast<double *>(lds_raw));
    }

    template <typename A>
    static __device__ __forceinline__ void readout(const A &a, const C (&v)[NR], uint64_t base, uint64_t dtid,
                                                   Readout ro, double *red)
    {
        const uint32_t tid = threadIdx.x;
        double nrm = 0.0, z = 0.0;
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            const uint64_t phys = base + dtid + slot_offset(a, j);
            const double re = (double)v[j].x, im = (double)v[j].y, p = re * re + im * im;
            nrm += p;
            z += ((phys >> ro.zpos) & 1ull) ? -p : p;
        }
        __syncthreads();  // the tile buffer is reused for the reduction
        red[tid] = nrm;
        red[NT + tid] = z;
        __syncthreads();
#pragma unroll
        for (int w = NT / 2; w > 0; w >>= 1) {
            if ((int)tid < w) {
                red[tid] += red[tid + w];
                red[NT + tid] += red[NT + tid + w];
            }
            __syncthreads();
        }
        if (tid == 0) {
            ro.out[0] = red[0];
            ro.out[1] = red[NT];
        }
    }
};

template <typename R, int LOG_NT, int LOG_R>
__global__ __launch_bounds__(1 << LOG_NT) void k_tile(TileArgs a)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    TileKernel<R, LOG_NT, LOG_R>::run(a, lds_raw, blockIdx.x, {nullptr, 0});
}

template <typename R, int LOG_NT, int LOG_R>
void launch_tile_inst(const TileArgs &a, uint64_t n_tiles, hipStream_t st)
{
    using C = typename Cx<R>::T;
    constexpr size_t bytes = sizeof(C) << (LOG_NT + LOG_R);
    // launches above the default dynamic LDS limit need the attribute first
    static bool attr_set = bytes <= 65536;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_tile<R, LOG_NT, LOG_R>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess)
            fail(QS_ERR_HIP, std::string("tile kernel attribute: ") + hipGetErrorString(e));
        attr_set = true;
    }
    if (n_tiles > 0x7fffffffull)
        fail(QS_ERR_UNSUPPORTED, "too many tiles for one launch");
    hipLaunchKernelGGL((k_tile<R, LOG_NT, LOG_R>), dim3((unsigned)n_tiles), dim3(1 << LOG_NT), bytes, st, a);
    check_launch("tile pass");
}

// Dispatch over the instantiated shapes: 2^6..2^10 threads, 2..32 amplitudes
// per thread, tile bytes within the LDS of one CU.
template <typename R>
void launch_tile_t(const TileArgs &a, uint64_t n_tiles, int log_r, int log_nt, hipStream_t st)
{
#define QS_TILE_CASE(NTB, RB)                                          \
    if (log_nt == NTB && log_r == RB) {                                \
        if constexpr ((sizeof(typename Cx<R>::T) << (NTB + RB)) <= 131072) { \
            launch_tile_inst<R, NTB, RB>(a, n_tiles, st);              \
            return;                                                    \
        }                                                              \
    }
#define QS_TILE_ROW(NTB) \
    QS_TILE_CASE(NTB, 1) QS_TILE_CASE(NTB, 2) QS_TILE_CASE(NTB, 3) QS_TILE_CASE(NTB, 4) QS_TILE_CASE(NTB, 5)
    QS_TILE_ROW(6)
    QS_TILE_ROW(7)
    QS_TILE_ROW(8)
    QS_TILE_ROW(9)
    QS_TILE_ROW(10)
#undef QS_TILE_ROW
#undef QS_TILE_CASE
    fail(QS_ERR_UNSUPPORTED, "tile shape not instantiated (log_nt=" + std::to_string(log_nt) +
                                 ", log_r=" + std::to_string(log_r) + ")");
}

}  // namespace qsim
