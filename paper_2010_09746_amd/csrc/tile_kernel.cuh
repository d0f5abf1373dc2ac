// Fused tile pass: a workgroup takes tiles of 2^K amplitudes one after the
// other, applies a run of gates that act on the tile's qubits to each, and
// stores each tile back in place.
//
// The tile is the set of amplitudes whose physical index has fixed bits
// outside K chosen positions pos[0..K) (the local qubits of the permutation
// pass, paper, Section 3).  With pos = 0..K-1 the tile is a contiguous block;
// when the pass only relabels qubits the tile gathers strided runs.
//
// Register layout: slot j of a thread holds the amplitude whose tile-local
// index is tbase | off(j ^ fl).  off deposits the slot bits into the LOG_R
// register tile bits chosen by the last OP_REMAP, tbase deposits the thread
// id into the other tile bits, and fl records exchanges (X) that were the
// same for the whole tile and were applied by relabelling slots instead of
// moving data.
//
// Data path per tile:
//   HBM -> registers  straight into the layout of the first OP_REMAP when
//                     the thread bits of that layout cover the lowest tile
//                     bits (runs of at least 128 contiguous bytes); otherwise
//                     into the plain layout (tile-local index j * NT + tid),
//                     which the first OP_REMAP moves
//   LDS <-> registers each OP_REMAP writes the tile to LDS at its tile-local
//                     indices and reads it back in the new layout, one
//                     component (real parts, then imaginary parts) per round,
//                     so LDS holds half the tile
//   gates             one-qubit updates and exchanges on register bits run
//                     inside a thread.  A control on a register bit selects
//                     register pairs by a test that is uniform over the
//                     wavefront, a control on a thread bit selects per lane
//                     without branching, and a control outside the tile
//                     decides for the whole tile from its base index
//   registers -> HBM  straight from the last layout when its thread bits
//                     cover the lowest tile bits, else through LDS
// The pass kernel runs one workgroup per tile; the batching form's persistent
// workgroups load their next tile into a second register array while the
// current one is processed.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "common.cuh"

namespace qsim {

template <typename R, int LOG_NT, int LOG_R, bool HALF = true, bool STREAM = true> struct TileKernel {
    using C = typename Cx<R>::T;
    static constexpr int NT = 1 << LOG_NT, NR = 1 << LOG_R, K = LOG_NT + LOG_R;
    static constexpr uint32_t CB = sizeof(C);  // bytes per amplitude

    // Order the LDS accesses of different lanes.  A single wavefront issues its
    // LDS instructions in order, so only the compiler must be kept from
    // reordering them; several wavefronts wait for their LDS operations and
    // meet at a barrier.  Neither form waits for outstanding global loads, so
    // the prefetch of the next tile stays in flight.
    static __device__ __forceinline__ void lds_sync()
    {
        if constexpr (NT == 64)
            __asm__ __volatile__("" ::: "memory");
        else
            __asm__ __volatile__("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
    }

    // register slot pair (j, j | 2^S) for pair index jj
    template <int S> static constexpr int pair_lo(int jj)
    {
        return ((jj >> S) << (S + 1)) | (jj & ((1 << S) - 1));
    }

    // dense 2x2 on slot S, in place, every pair.  With SW the slot's pattern
    // bit is flipped (the upper slot of a pair holds pattern bit 0).
    template <int S, bool SW> static __device__ __forceinline__ void bfly(C (&v)[NR], const Mat<R> &m)
    {
#pragma unroll
        for (int jj = 0; jj < NR / 2; ++jj) {
            const int j = pair_lo<S>(jj), j1 = j | (1 << S);
            if (SW)
                m.apply(v[j1], v[j]);
            else
                m.apply(v[j], v[j1]);
        }
    }

    // Controlled 2x2.  A pair takes part when its register pattern has every
    // control slot set, (j & rm) == rv with rv = rm & ~fl (a scalar test), and,
    // with LANE, the lane has every control thread bit set (lp, a select).
    template <int S, bool SW, bool LANE>
    static __device__ __forceinline__ void bfly_c(C (&v)[NR], const Mat<R> &m, uint32_t rm, uint32_t rv, bool lp)
    {
#pragma unroll
        for (int jj = 0; jj < NR / 2; ++jj) {
            const int j = pair_lo<S>(jj), j0 = SW ? (j | (1 << S)) : j, j1 = SW ? j : (j | (1 << S));
            if (((uint32_t)j & rm) == rv) {
                if (LANE) {
                    C x = v[j0], y = v[j1];
                    m.apply(x, y);
                    v[j0].x = lp ? x.x : v[j0].x;
                    v[j0].y = lp ? x.y : v[j0].y;
                    v[j1].x = lp ? y.x : v[j1].x;
                    v[j1].y = lp ? y.y : v[j1].y;
                } else {
                    m.apply(v[j0], v[j1]);
                }
            }
        }
    }

    // exchange on slot S with any controls: scalar test per pair, lane select
    template <int S>
    static __device__ __forceinline__ void xswap_c(C (&v)[NR], uint32_t rm, uint32_t rv, bool lp)
    {
#pragma unroll
        for (int jj = 0; jj < NR / 2; ++jj) {
            const int j = pair_lo<S>(jj), j1 = j | (1 << S);
            if (((uint32_t)j & rm) == rv) {
                const C x = v[j], y = v[j1];
                v[j].x = lp ? y.x : x.x;
                v[j].y = lp ? y.y : x.y;
                v[j1].x = lp ? x.x : y.x;
                v[j1].y = lp ? x.y : y.y;
            }
        }
    }

    template <int S, bool SW>
    static __device__ __forceinline__ void apply_u(C (&v)[NR], const Mat<R> &m, uint32_t rm, uint32_t lm, uint32_t rv,
                                                   bool lp)
    {
        if ((rm | lm) == 0)
            bfly<S, SW>(v, m);
        else if (lm == 0)
            bfly_c<S, SW, false>(v, m, rm, rv, lp);
        else
            bfly_c<S, SW, true>(v, m, rm, rv, lp);
    }

    template <int S = 0>
    static __device__ __forceinline__ void dispatch_u(int slot, uint32_t sw, C (&v)[NR], const Mat<R> &m, uint32_t rm,
                                                      uint32_t lm, uint32_t rv, bool lp)
    {
        if (slot == S || S == LOG_R - 1) {
            if (sw)
                apply_u<S, true>(v, m, rm, lm, rv, lp);
            else
                apply_u<S, false>(v, m, rm, lm, rv, lp);
        } else if constexpr (S + 1 < LOG_R) {
            dispatch_u<S + 1>(slot, sw, v, m, rm, lm, rv, lp);
        }
    }

    template <int S = 0>
    static __device__ __forceinline__ void dispatch_x(int slot, C (&v)[NR], uint32_t rm, uint32_t lm, uint32_t rv,
                                                      bool lp)
    {
        if (slot == S || S == LOG_R - 1) {
            xswap_c<S>(v, rm, rv, lp);
        } else if constexpr (S + 1 < LOG_R) {
            dispatch_x<S + 1>(slot, v, rm, lm, rv, lp);
        }
    }

    // Two shears on one pair, in place: x += p y, then y += q x (with the new
    // x).  8 real multiply-adds, each reading the register it writes, so no
    // old value has to stay alive.
    static __device__ __forceinline__ void spair(C &x, C &y, R pr, R pi, R qr, R qi)
    {
        x.x = fmadd(pr, y.x, x.x);
        x.y = fmadd(pr, y.y, x.y);
        x.x = fmadd(-pi, y.y, x.x);
        x.y = fmadd(pi, y.x, x.y);
        y.x = fmadd(qr, x.x, y.x);
        y.y = fmadd(qr, x.y, y.y);
        y.x = fmadd(-qi, x.y, y.x);
        y.y = fmadd(qi, x.x, y.y);
    }
    // the shears on slot S, every pair.  With SW the slot's pattern bit is
    // flipped (the upper slot of a pair holds pattern bit 0).
    template <int S, bool SW> static __device__ __forceinline__ void sfly(C (&v)[NR], R pr, R pi, R qr, R qi)
    {
#pragma unroll
        for (int jj = 0; jj < NR / 2; ++jj) {
            const int j = pair_lo<S>(jj), j1 = j | (1 << S);
            if (SW)
                spair(v[j1], v[j], pr, pi, qr, qi);
            else
                spair(v[j], v[j1], pr, pi, qr, qi);
        }
    }
    template <int S = 0>
    static __device__ __forceinline__ void dispatch_shear(int slot, uint32_t sw, C (&v)[NR], R pr, R pi, R qr, R qi)
    {
        if (slot == S || S == LOG_R - 1) {
            if (sw)
                sfly<S, true>(v, pr, pi, qr, qi);
            else
                sfly<S, false>(v, pr, pi, qr, qi);
        } else if constexpr (S + 1 < LOG_R) {
            dispatch_shear<S + 1>(slot, sw, v, pr, pi, qr, qi);
        }
    }

    // multiply by (pr, pi) the amplitudes whose pattern bit of slot S is 1
    // (the slot bit itself with SW clear, its complement with SW set)
    template <int S, bool SW> static __device__ __forceinline__ void phase_slots(C (&v)[NR], R pr, R pi)
    {
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            if (((j >> S) & 1) != (SW ? 1 : 0)) {
                const R x = v[j].x;
                v[j].x = fmadd(pr, x, -pi * v[j].y);
                v[j].y = fmadd(pr, v[j].y, pi * x);
            }
        }
    }
    template <int S = 0>
    static __device__ __forceinline__ void dispatch_phase(int slot, uint32_t sw, C (&v)[NR], R pr, R pi)
    {
        if (slot == S || S == LOG_R - 1) {
            if (sw)
                phase_slots<S, true>(v, pr, pi);
            else
                phase_slots<S, false>(v, pr, pi);
        } else if constexpr (S + 1 < LOG_R) {
            dispatch_phase<S + 1>(slot, sw, v, pr, pi);
        }
    }

    // Exchange register slot bit S with lane bit 4 (L5 false) or 5 (L5 true)
    // of the wavefront: for each register pair (a, b) of the slot, the lanes
    // of a whose lane bit is 1 trade places with the lanes of b whose lane
    // bit is 0 (v_permlane16_swap / v_permlane32_swap, one instruction per
    // 32-bit word, no LDS).  With SW the slot's pattern bit is flipped: the
    // pair is taken the other way round, and the flip stays.
    template <bool L5> static __device__ __forceinline__ void swap_words(uint32_t &a, uint32_t &b)
    {
        if constexpr (L5) {
            const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
            a = r[0];
            b = r[1];
        } else {
            const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
            a = r[0];
            b = r[1];
        }
    }
    template <bool L5> static __device__ __forceinline__ void swap_real(R &a, R &b)
    {
        if constexpr (sizeof(R) == 8) {
            auto x = __builtin_bit_cast(uint2, a);
            auto y = __builtin_bit_cast(uint2, b);
            swap_words<L5>(x.x, y.x);
            swap_words<L5>(x.y, y.y);
            a = __builtin_bit_cast(R, x);
            b = __builtin_bit_cast(R, y);
        } else {
            uint32_t x = __builtin_bit_cast(uint32_t, a), y = __builtin_bit_cast(uint32_t, b);
            swap_words<L5>(x, y);
            a = __builtin_bit_cast(R, x);
            b = __builtin_bit_cast(R, y);
        }
    }
    template <int S, bool L5, bool SW> static __device__ __forceinline__ void lane_swap(C (&v)[NR])
    {
#pragma unroll
        for (int jj = 0; jj < NR / 2; ++jj) {
            const int j = pair_lo<S>(jj), j1 = j | (1 << S);
            C &a = SW ? v[j1] : v[j];
            C &b = SW ? v[j] : v[j1];
            swap_real<L5>(a.x, b.x);
            swap_real<L5>(a.y, b.y);
        }
    }
    template <int S = 0>
    static __device__ __forceinline__ void dispatch_lane_swap(int slot, bool l5, uint32_t sw, C (&v)[NR])
    {
        if (slot == S || S == LOG_R - 1) {
            if (l5)
                sw ? lane_swap<S, true, true>(v) : lane_swap<S, true, false>(v);
            else
                sw ? lane_swap<S, false, true>(v) : lane_swap<S, false, false>(v);
        } else if constexpr (S + 1 < LOG_R) {
            dispatch_lane_swap<S + 1>(slot, l5, sw, v);
        }
    }

    // One-qubit 2x2 on thread bit B < 4 (a lane bit of the wavefront), every
    // register amplitude: each lane reads the amplitude of lane tid ^ 2^B by
    // DPP moves within rows of 16 lanes (one quad permutation for bits 0 and
    // 1; a half-row mirror, XOR 7, and the quad permutation XOR 3 for bit 2;
    // a row mirror, XOR 15, and a half-row mirror for bit 3), one or two per
    // 32-bit word, and the lane whose bit is b computes row b of the matrix:
    // own M[b][b] + partner M[b][1-b] (c: the lane's two coefficients).
    template <int B> static __device__ __forceinline__ uint32_t xor_lane_word(uint32_t w)
    {
        const int x = (int)w;
        if constexpr (B == 0)
            return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, true);
        else if constexpr (B == 1)
            return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, true);
        else if constexpr (B == 2)
            return (uint32_t)__builtin_amdgcn_mov_dpp(__builtin_amdgcn_mov_dpp(x, 0x141, 0xF, 0xF, true), 0x1B, 0xF,
                                                      0xF, true);
        else
            return (uint32_t)__builtin_amdgcn_mov_dpp(__builtin_amdgcn_mov_dpp(x, 0x140, 0xF, 0xF, true), 0x141, 0xF,
                                                      0xF, true);
    }
    template <int B> static __device__ __forceinline__ R xor_lane(R a)
    {
        if constexpr (sizeof(R) == 8) {
            auto w = __builtin_bit_cast(uint2, a);
            w.x = xor_lane_word<B>(w.x);
            w.y = xor_lane_word<B>(w.y);
            return __builtin_bit_cast(R, w);
        } else {
            return __builtin_bit_cast(R, xor_lane_word<B>(__builtin_bit_cast(uint32_t, a)));
        }
    }
    template <int B> static __device__ __forceinline__ void lane_gate(C (&v)[NR], const R (&c)[4])
    {
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            const R px = xor_lane<B>(v[j].x), py = xor_lane<B>(v[j].y);
            const R ox = v[j].x, oy = v[j].y;
            v[j].x = fmadd(c[0], ox, fmadd(-c[1], oy, fmadd(c[2], px, -c[3] * py)));
            v[j].y = fmadd(c[0], oy, fmadd(c[1], ox, fmadd(c[2], py, c[3] * px)));
        }
    }
    static __device__ __forceinline__ void dispatch_lane_gate(uint32_t b, uint32_t tid, C (&v)[NR], const double *m)
    {
        const bool hi = ((tid >> b) & 1u) != 0;
        const R c[4] = {(R)(hi ? m[6] : m[0]), (R)(hi ? m[7] : m[1]), (R)(hi ? m[4] : m[2]), (R)(hi ? m[5] : m[3])};
        if (b == 0)
            lane_gate<0>(v, c);
        else if (b == 1)
            lane_gate<1>(v, c);
        else if (b == 2)
            lane_gate<2>(v, c);
        else
            lane_gate<3>(v, c);
    }

    // flip the sign bit where sg has it set (sg is 0 or the sign mask)
    static __device__ __forceinline__ R flip_sign(R x, uint32_t sg)
    {
        if constexpr (sizeof(R) == 8)
            return __builtin_bit_cast(R, __builtin_bit_cast(uint64_t, x) ^ ((uint64_t)sg << 32));
        else
            return __builtin_bit_cast(R, __builtin_bit_cast(uint32_t, x) ^ sg);
    }

    // LDS byte offsets (EB times lds_swizzle of the tile bit) of the register
    // slot bits of a layout: uniform values, shipped by the lowering with
    // each re-layout
    struct SlotOffs {
        uint32_t o[LOG_R];
    };
    // from the record's LDS slots; opaque to the compiler, so that the
    // addresses stay one XOR of a thread part and a scalar per slot (it
    // otherwise moves the scaling into every address)
    static __device__ __forceinline__ SlotOffs offs_of(const uint32_t *w)
    {
        SlotOffs so;
#pragma unroll
        for (int q = 0; q < LOG_R; ++q) {
            so.o[q] = w[q] * EB;
            __asm__("" : "+s"(so.o[q]));
        }
        return so;
    }

    // Visit the slots j in Gray-code order with the XOR over the set bits s of
    // j of basis(s): consecutive slots differ in one bit, so each value costs
    // one XOR and only one is live at a time.
    template <typename T, typename B, typename Fn>
    static __device__ __forceinline__ void for_slots(B basis, Fn fn)
    {
        T acc = 0;
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            if (i)
                acc ^= basis(__builtin_ctz(i));
            fn(i ^ (i >> 1), acc);
        }
    }

    // the thread id deposited into tile bits: thread bit i goes to tile bit
    // (map >> 4i) & 15 (the lane map of an OP_REMAP)
    static __device__ __forceinline__ uint32_t lane_bits(uint64_t map, uint32_t tid)
    {
        uint32_t tb = 0;
#pragma unroll
        for (int i = 0; i < LOG_NT; ++i)
            tb |= ((tid >> i) & 1u) << ((map >> (4 * i)) & 15u);
        return tb;
    }

    // the thread id deposited into physical positions: thread bit i goes to lane[i]
    template <typename P> static __device__ __forceinline__ uint64_t lane_offset(P lane, uint32_t tid)
    {
        uint64_t d = 0;
#pragma unroll
        for (int i = 0; i < LOG_NT; ++i)
            d |= (uint64_t)((tid >> i) & 1u) << lane[i];
        return d;
    }

    // the tile number with a zero inserted at every tile position (ascending)
    template <typename A> static __device__ __forceinline__ uint64_t tile_base(const A &a, uint64_t tile)
    {
        uint64_t base = tile;
#pragma unroll
        for (int b = 0; b < K; ++b) {
            const int p = a.pos[b];
            base = ((base >> p) << (p + 1)) | (base & ((1ull << p) - 1));
        }
        return base;
    }

    // LDS holds one component (real or imaginary part) of the tile at a time:
    // half the bytes of the tile, so that more workgroups fit a CU.  The
    // read-out reduction needs 2 NT doubles.
    // With HALF a re-layout moves one component per round and LDS holds half
    // the tile; otherwise one round moves whole amplitudes (fewer barriers,
    // for kernels whose residency LDS does not limit).
    static constexpr uint32_t RB = sizeof(R);
    static constexpr uint32_t EB = HALF ? RB : CB;  // bytes per LDS element of a re-layout
    static constexpr uint32_t LDS_BYTES = (EB << K) > 16u * NT ? (EB << K) : 16u * NT;
    // the plain layout: thread bits are tile bits 0..LOG_NT-1, slot bit s is
    // tile bit LOG_NT + s
    static __device__ __forceinline__ SlotOffs offs_plain()
    {
        SlotOffs so;
#pragma unroll
        for (int s = 0; s < LOG_R; ++s)
            so.o[s] = swz(1u << (LOG_NT + s)) * EB;
        return so;
    }

    // element COMP of an amplitude in LDS: 0 real part, 1 imaginary part, 2
    // both (a two-element vector, one LDS access)
    using V2 = R __attribute__((ext_vector_type(2)));
    template <int COMP> static __device__ __forceinline__ void put(uint32_t addr, const C &c)
    {
        if constexpr (COMP == 0)
            *at<R>(addr) = c.x;
        else if constexpr (COMP == 1)
            *at<R>(addr) = c.y;
        else
            *at<V2>(addr) = V2{c.x, c.y};
    }
    template <int COMP> static __device__ __forceinline__ void get(uint32_t addr, C &c)
    {
        if constexpr (COMP == 0) {
            c.x = *at<R>(addr);
        } else if constexpr (COMP == 1) {
            c.y = *at<R>(addr);
        } else {
            const V2 t = *at<V2>(addr);
            c.x = t.x;
            c.y = t.y;
        }
    }

    // LDS slot of tile-local index i (lds_swizzle): thread bits placed on
    // high tile bits by a re-layout send a wavefront's lanes to different
    // banks instead of one.
    static __host__ __device__ __forceinline__ constexpr uint32_t swz(uint32_t i) { return lds_swizzle(i, K); }

    // LDS address of the buffer.  The kernels that use TileKernel have no
    // static LDS (checked at launch), so the buffer starts at LDS address 0
    // and a byte offset below LDS_BYTES can be XORed into it instead of added
    // (an address is then one XOR of a per-thread and a per-slot part).
    static __device__ __forceinline__ uint32_t lds_base(const unsigned char *lds)
    {
        return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) unsigned char *)lds;
    }
    template <typename T = R> static __device__ __forceinline__ __attribute__((address_space(3))) T *at(uint32_t addr)
    {
        return (__attribute__((address_space(3))) T *)(uintptr_t)addr;
    }

    // element COMP of every amplitude, registers <-> LDS at the tile-local
    // indices of the layout (tbase, so, fl)
    template <int COMP>
    static __device__ __forceinline__ void to_lds(unsigned char *lds, C (&v)[NR], uint32_t tbase, const SlotOffs &so,
                                                   uint32_t fl)
    {
        uint32_t fo = 0;  // the flipped slot bits of the pattern
#pragma unroll
        for (int s = 0; s < LOG_R; ++s)
            fo ^= ((fl >> s) & 1u) ? so.o[s] : 0u;
        const uint32_t tb = lds_base(lds) ^ (swz(tbase) * EB) ^ fo;
        for_slots<uint32_t>([&](int s) { return so.o[s]; },
                            [&](int j, uint32_t o) { put<COMP>(tb ^ o, v[j]); });
    }
    template <int COMP>
    static __device__ __forceinline__ void from_lds(const unsigned char *lds, C (&v)[NR], uint32_t tbase,
                                                     const SlotOffs &so)
    {
        const uint32_t tb = lds_base(lds) ^ (swz(tbase) * EB);
        for_slots<uint32_t>([&](int s) { return so.o[s]; },
                            [&](int j, uint32_t o) { get<COMP>(tb ^ o, v[j]); });
    }

    // Re-layout (tbase, so, fl) -> (tbase2, so2, no flips) through LDS, one
    // component per round with HALF.
    // With wave_local the two layouts put the same tile bits on the
    // wavefront-index bits of the thread id: each wavefront reads back only
    // LDS slots it wrote, in order, so only the compiler is kept from
    // reordering the accesses.  Every other re-layout ends with a barrier, so
    // a wavefront-local one never overlaps another wavefront's reads of the
    // slots it writes.
    static __device__ __forceinline__ void relayout(unsigned char *lds, C (&v)[NR], uint32_t tbase,
                                                    const SlotOffs &so, uint32_t fl, uint32_t tbase2,
                                                    const SlotOffs &so2, bool wave_local = false)
    {
        auto sync = [&] {
            if (wave_local)
                __asm__ __volatile__("" ::: "memory");
            else
                lds_sync();
        };
        if constexpr (HALF) {
            to_lds<0>(lds, v, tbase, so, fl);
            sync();
            from_lds<0>(lds, v, tbase2, so2);
            sync();
            to_lds<1>(lds, v, tbase, so, fl);
            sync();
            from_lds<1>(lds, v, tbase2, so2);
            sync();
        } else {
            to_lds<2>(lds, v, tbase, so, fl);
            sync();
            from_lds<2>(lds, v, tbase2, so2);
            sync();
        }
    }

    using OpPtr = const __attribute__((address_space(4))) TileOp *;

    // the fields of one operation, read together (scalar registers)
    struct OpV {
        int32_t kind, slot;
        uint32_t rmask, lmask, tlane, aux;
        uint64_t hmask, hbit;
        double m[8];
        uint32_t w[6];  // the first words of m (OP_REMAP: LDS slots of the new layout's slot bits)
    };
    // The record as three wide scalar loads (64 + 32 + 8 bytes) issued
    // together, so that one wait covers the whole operation.
    using U16 = uint32_t __attribute__((ext_vector_type(16)));
    using U8 = uint32_t __attribute__((ext_vector_type(8)));
    using U2 = uint32_t __attribute__((ext_vector_type(2)));
    static __device__ __forceinline__ OpV fetch(OpPtr ops, int i)
    {
        using CP = const __attribute__((address_space(4))) unsigned char *;
        const CP p = (CP)(ops + i);
        const U16 a = *(const __attribute__((address_space(4))) U16 *)p;
        const U8 b = *(const __attribute__((address_space(4))) U8 *)(p + 64);
        const U2 c = *(const __attribute__((address_space(4))) U2 *)(p + 96);
        __asm__ __volatile__("" ::"s"(a), "s"(b), "s"(c));
        auto d = [](uint32_t lo, uint32_t hi) { return __builtin_bit_cast(double, (uint64_t)lo | ((uint64_t)hi << 32)); };
        OpV o;
        o.kind = (int32_t)a[0];
        o.slot = (int32_t)a[1];
        o.rmask = a[2];
        o.lmask = a[3];
        o.tlane = a[4];
        o.aux = a[5];
        o.hmask = (uint64_t)a[6] | ((uint64_t)a[7] << 32);
        o.hbit = (uint64_t)a[8] | ((uint64_t)a[9] << 32);
        o.m[0] = d(a[10], a[11]);
        o.m[1] = d(a[12], a[13]);
        o.m[2] = d(a[14], a[15]);
        o.m[3] = d(b[0], b[1]);
        o.m[4] = d(b[2], b[3]);
        o.m[5] = d(b[4], b[5]);
        o.m[6] = d(b[6], b[7]);
        o.m[7] = d(c[0], c[1]);
#pragma unroll
        for (int q = 0; q < 6; ++q)
            o.w[q] = a[10 + q];
        return o;
    }

    // Per-tile read-out of the final amplitudes: sum |a|^2 and sum |a|^2 (1 - 2 b)
    // where b is the bit at physical position zpos (the first qubit), reduced
    // over the workgroup in a fixed order and written to out[0..1].
    struct Readout {
        double *out;  // NULL: none; else two doubles per tile, tile t at out + 2 (t - t_first) / t_step
        int zpos;
    };

    // Tiles t_first, t_first + t_step, ... below t_end.  A is TileArgs, read
    // from kernel arguments or from device memory.  With BASIS, a pass whose
    // TileArgs::io has bit 4 set reads nothing: its tiles start as the basis
    // state |0...0> (1 at physical index 0, 0 elsewhere).
    // With ZB each tile t also writes NV = 1 + LOG_R + LOG_NT doubles, value v
    // at zparts[v * zstride + t]: the
    // sum of |a|^2 over the tile, then for each register slot bit and each
    // thread-id bit of the store layout (positions st_reg, st_lane) the sum of
    // |a|^2 over the amplitudes whose bit there is 1, reduced in a fixed order
    // (wavefront butterflies, then the wavefronts in order).
    static constexpr int NV = 1 + LOG_R + LOG_NT;
    template <bool PF, bool BASIS = false, bool ZB = false, typename A>
    static __device__ __forceinline__ void run_range(const A &a, unsigned char *lds, uint64_t t_first, uint64_t t_end,
                                                     uint64_t t_step, Readout ro, double *zparts = nullptr,
                                                     uint64_t zstride = 0)
    {
        C *st = reinterpret_cast<C *>(a.state);
        OpPtr ops = (OpPtr)(a.ops);
        const uint32_t tid = threadIdx.x;
        const int n_ops = a.n_ops;
        const bool dload = (a.io & 1u) != 0, dstore = (a.io & 2u) != 0;

        // Load and store layouts: a thread's offset plus, per slot, the XOR
        // over its set bits of the slot bits' position bits.
        const uint64_t lane_ld = lane_offset(a.ld_lane, tid);
        const uint64_t lane_st = lane_offset(a.st_lane, tid);
        auto pbit_ld = [&](int s) { return 1ull << a.ld_reg[s]; };
        auto pbit_st = [&](int s) { return 1ull << a.st_reg[s]; };

        // v holds the tile being processed; the next tile of the workgroup is
        // loaded into w while v is processed and moves into v after v's
        // stores are issued, so the wait for it never waits for those stores
        C v[NR];
        auto load = [&](C(&dst)[NR], uint64_t tile) {
            const C *src = st + tile_base(a, tile) + lane_ld;
            if constexpr (BASIS) {
                if (a.io & 16u) {
                    const bool origin = (src == st);
                    for_slots<uint64_t>(pbit_ld, [&](int j, uint64_t o) {
                        dst[j].x = (origin && o == 0) ? R(1) : R(0);
                        dst[j].y = R(0);
                    });
                    return;
                }
            }
            // with STREAM (one pass over an HBM-resident state, every amplitude
            // read once and written once, whole 128-byte lines per access)
            // loads and stores are non-temporal: +3-6% bandwidth on passes
            // with few gates
            for_slots<uint64_t>(pbit_ld, [&](int j, uint64_t o) {
                if constexpr (STREAM) {
                    dst[j].x = __builtin_nontemporal_load(&src[o].x);
                    dst[j].y = __builtin_nontemporal_load(&src[o].y);
                } else {
                    dst[j] = src[o];
                }
            });
        };
        if constexpr (PF) {
            if (t_first < t_end)
                load(v, t_first);
            // wait for the first tile here, so that the loop's own waits are only
            // those for the prefetched tile (vmcnt(0): expcnt and lgkmcnt left at
            // their maxima)
            __builtin_amdgcn_s_waitcnt(0x0F70);
        }

        for (uint64_t t = t_first; t < t_end; t += t_step) {
            C w[NR];
            const bool more = PF && t + t_step < t_end;
            if constexpr (!PF) {
                load(v, t);
                __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0), as above
            } else if (more)
                load(w, t + t_step);
            const uint64_t base = tile_base(a, t);

            SlotOffs so = offs_plain();
            uint32_t tbase = 0, fl = 0;
            bool have = false;
            int oi = 0;
            if (dload) {
                const OpV first = fetch(ops, 0);
                so = offs_of(first.w);
                tbase = lane_bits(first.hbit, tid);
                have = true;
                oi = 1;
            } else if (n_ops > 0) {
                // loaded in the plain layout; the first OP_REMAP moves it
                tbase = tid;
                have = true;
            }

            for (; oi < n_ops; ++oi) {
                const OpV cur = fetch(ops, oi);
                const int kind = cur.kind;
                // the most frequent operations first: shears have no controls
                static_assert((OP_SHEAR | 2) == OP_SHEAR2, "one test for both shear records");
                if ((kind | 2) == OP_SHEAR2) {
                    const int slot = cur.slot;
                    fl ^= cur.tlane ? 1u << slot : 0u;
                    dispatch_shear(slot, (fl >> slot) & 1u, v, (R)cur.m[0], (R)cur.m[1], (R)cur.m[2], (R)cur.m[3]);
                    if (kind == OP_SHEAR2) {
                        const int s2 = (int)(cur.aux & 255u);
                        fl ^= (cur.aux >> 8) ? 1u << s2 : 0u;
                        dispatch_shear(s2, (fl >> s2) & 1u, v, (R)cur.m[4], (R)cur.m[5], (R)cur.m[6], (R)cur.m[7]);
                    }
                } else if (kind == OP_REMAP) {
                    const SlotOffs so2 = offs_of(cur.w);
                    const uint32_t tbase2 = lane_bits(cur.hbit, tid);
                    relayout(lds, v, tbase, so, fl, tbase2, so2, (cur.aux & REMAP_WAVE_LOCAL) != 0);
                    so = so2;
                    tbase = tbase2;
                    fl = 0;
                } else if (kind == OP_LSWAP) {
                    // slot bit `slot` <-> lane bit tlane; the tile bit lmask
                    // moves into the slot, the tile bit rmask onto the lane
                    const int slot = cur.slot;
                    dispatch_lane_swap(slot, cur.tlane == 5, (fl >> slot) & 1u, v);
                    tbase = (tbase & ~cur.lmask) | (((tid >> cur.tlane) & 1u) ? cur.rmask : 0u);
                    const uint32_t o_new = offs_of(cur.w).o[0];
#pragma unroll
                    for (int q = 0; q < LOG_R; ++q)
                        so.o[q] = q == slot ? o_new : so.o[q];
                } else if (kind == OP_LANE) {
                    dispatch_lane_gate(cur.tlane, tid, v, cur.m);
                } else if ((base & cur.hmask) == cur.hmask) {
                    const uint32_t rm = cur.rmask, lm = cur.lmask;
                    const uint32_t rv = rm & ~fl;
                    const bool lp = (tbase & lm) == lm;
                    const int slot = cur.slot;
                    if (kind == OP_PHASE) {
                        dispatch_phase(slot, (fl >> slot) & 1u, v, (R)cur.m[0], (R)cur.m[1]);
                    } else if (kind == OP_U) {
                        Mat<R> m;
#pragma unroll
                        for (int q = 0; q < 8; ++q)
                            m.a[q] = (R)cur.m[q];
                        dispatch_u(slot, (fl >> slot) & 1u, v, m, rm, lm, rv, lp);
                    } else if (kind == OP_X) {
                        if ((rm | lm) == 0) {
                            fl ^= 1u << slot;
                        } else {
                            dispatch_x(slot, v, rm, lm, rv, lp);
                        }
                    } else if (kind == OP_NEG) {
                        // sign flips: the slot test is scalar, the lane test a mask
                        const uint32_t sg = lp ? 0x80000000u : 0u;
#pragma unroll
                        for (int j = 0; j < NR; ++j) {
                            const uint32_t sj = ((uint32_t)j & rm) == rv ? sg : 0u;
                            v[j].x = flip_sign(v[j].x, sj);
                            v[j].y = flip_sign(v[j].y, sj);
                        }
                    } else {  // OP_DIAG: target on register slot `slot`, thread bit tlane, or outside (hbit)
                        R d0r = (R)cur.m[0], d0i = (R)cur.m[1], d1r = (R)cur.m[2], d1i = (R)cur.m[3];
                        // lanes outside the thread-bit controls multiply by 1
                        d0r = lp ? d0r : (R)1;
                        d0i = lp ? d0i : (R)0;
                        d1r = lp ? d1r : (R)1;
                        d1i = lp ? d1i : (R)0;
                        const bool lsel = cur.tlane ? (tbase & cur.tlane) != 0 : (base & cur.hbit) != 0;
                        const R lr = lsel ? d1r : d0r, li = lsel ? d1i : d0i;
#pragma unroll
                        for (int j = 0; j < NR; ++j) {
                            if (((uint32_t)j & rm) == rv) {
                                R dr = lr, di = li;
                                if (slot >= 0) {
                                    const bool sl = ((((uint32_t)j ^ fl) >> slot) & 1u) != 0;
                                    dr = sl ? d1r : d0r;
                                    di = sl ? d1i : d0i;
                                }
                                const C x = v[j];
                                v[j].x = fmadd(dr, x.x, -di * x.y);
                                v[j].y = fmadd(dr, x.y, di * x.x);
                            }
                        }
                    }
                }
            }

            // Store.  Direct: slot j holds pattern j ^ fl of the last layout,
            // whose offset is the slot's offset XOR the flipped bits' offset.
            const bool direct = have && dstore;
            if (a.io & 4u) {
                // bit permutation of the tile (no ops ran, so v is in tile-index
                // order j * NT + tid): the permutation is linear, so a lane part
                // and per-slot parts are XORed
                uint32_t pl = 0;
#pragma unroll
                for (int i = 0; i < LOG_NT; ++i)
                    pl |= ((tid >> i) & 1u) << a.sperm[i];
                // one component per round; LDS slots as in to_lds
                const uint32_t wl = lds_base(lds) ^ (swz(pl) * RB), rl = lds_base(lds) ^ (swz(tid) * RB);
                for_slots<uint32_t>([&](int s) { return swz(1u << a.sperm[LOG_NT + s]) * RB; },
                                    [&](int j, uint32_t o) { *at(wl ^ o) = v[j].x; });
                lds_sync();
#pragma unroll
                for (int j = 0; j < NR; ++j)
                    v[j].x = *at(rl ^ (swz((uint32_t)j << LOG_NT) * RB));
                lds_sync();
                for_slots<uint32_t>([&](int s) { return swz(1u << a.sperm[LOG_NT + s]) * RB; },
                                    [&](int j, uint32_t o) { *at(wl ^ o) = v[j].y; });
                lds_sync();
#pragma unroll
                for (int j = 0; j < NR; ++j)
                    v[j].y = *at(rl ^ (swz((uint32_t)j << LOG_NT) * RB));
            } else if (have && !dstore) {
                relayout(lds, v, tbase, so, fl, tid, offs_plain());
            }
            uint64_t dfl = 0;
            if (direct) {
#pragma unroll
                for (int s = 0; s < LOG_R; ++s)
                    dfl ^= ((fl >> s) & 1u) ? pbit_st(s) : 0ull;
            }
            C *dst = st + base + lane_st;
            double nrm = 0.0, z = 0.0;
            double zt = 0.0, zu[LOG_R];
#pragma unroll
            for (int q = 0; q < LOG_R; ++q)
                zu[q] = 0.0;
            for_slots<uint64_t>(pbit_st, [&](int j, uint64_t o) {
                if constexpr (STREAM) {
                    __builtin_nontemporal_store(v[j].x, &dst[o ^ dfl].x);
                    __builtin_nontemporal_store(v[j].y, &dst[o ^ dfl].y);
                } else {
                    dst[o ^ dfl] = v[j];
                }
                if constexpr (ZB) {
                    const double re = (double)v[j].x, im = (double)v[j].y, p = re * re + im * im;
                    zt += p;
#pragma unroll
                    for (int q = 0; q < LOG_R; ++q)
                        if ((j >> q) & 1)
                            zu[q] += p;
                }
                if (ro.out) {
                    const uint64_t phys = base + lane_st + (o ^ dfl);
                    const double re = (double)v[j].x, im = (double)v[j].y, p = re * re + im * im;
                    nrm += p;
                    z += ((phys >> ro.zpos) & 1ull) ? -p : p;
                }
            });
            if (ro.out)
                reduce_pair(nrm, z, ro.out + 2 * ((t - t_first) / t_step), reinterpret_cast<double *>(lds));
            if constexpr (ZB)
                reduce_bits(zt, zu, direct ? fl : 0u, zparts + t, zstride, reinterpret_cast<double *>(lds));
            lds_sync();  // the next tile reuses the LDS buffer
            if constexpr (PF) {
                if (more) {
#pragma unroll
                    for (int j = 0; j < NR; ++j)
                        v[j] = w[j];
                }
            }
        }
    }

    // The NV sums of the ZB read-out: slot bit q holds 1 where (j >> q) ^ (flips
    // >> q) is 1 (a slot whose exchange was applied by relabelling counts the
    // other half), thread bit i where the thread id has it.
    static __device__ __forceinline__ void reduce_bits(double zt, const double (&zu)[LOG_R], uint32_t flips,
                                                       double *out, uint64_t stride, double *red)
    {
        const uint32_t tid = threadIdx.x;
        double zv[NV];
        zv[0] = zt;
#pragma unroll
        for (int q = 0; q < LOG_R; ++q)
            zv[1 + q] = ((flips >> q) & 1u) ? zt - zu[q] : zu[q];
#pragma unroll
        for (int i = 0; i < LOG_NT; ++i)
            zv[1 + LOG_R + i] = ((tid >> i) & 1u) ? zt : 0.0;
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1)
                zv[v] += __shfl_xor(zv[v], d);
        // other wavefronts may still read LDS slots of a wavefront-local re-layout
        lds_sync();
        if ((tid & 63u) == 0) {
#pragma unroll
            for (int v = 0; v < NV; ++v)
                red[(tid >> 6) * NV + v] = zv[v];
        }
        lds_sync();
        if (tid < (uint32_t)NV) {
            double r = 0.0;
            for (int w = 0; w < (NT >> 6); ++w)
                r += red[w * NV + tid];
            out[stride * tid] = r;
        }
    }

    // Sum nrm and z over the workgroup in a fixed order; thread 0 writes out[0..1].
    static __device__ __forceinline__ void reduce_pair(double nrm, double z, double *out, double *red)
    {
        const uint32_t tid = threadIdx.x;
        lds_sync();
        red[tid] = nrm;
        red[NT + tid] = z;
        lds_sync();
#pragma unroll
        for (int w = NT / 2; w > 0; w >>= 1) {
            if ((int)tid < w) {
                red[tid] += red[tid + w];
                red[NT + tid] += red[NT + tid + w];
            }
            lds_sync();
        }
        if (tid == 0) {
            out[0] = red[0];
            out[1] = red[NT];
        }
        lds_sync();
    }
};

// TileKernel XORs byte offsets into the LDS base address, which needs the
// dynamic LDS buffer to start at LDS address 0: no static LDS in the kernel.
inline void check_no_static_lds(const void *fn, const char *what)
{
    hipFuncAttributes fa{};
    hipError_t e = hipFuncGetAttributes(&fa, fn);
    if (e != hipSuccess)
        fail(QS_ERR_HIP, std::string(what) + " attributes: " + hipGetErrorString(e));
    if (fa.sharedSizeBytes != 0)
        fail(QS_ERR_UNSUPPORTED, std::string(what) + " has static LDS; its LDS addressing assumes none");
}

// One workgroup per tile.  (A persistent grid that prefetches the next tile,
// with or without staggered starts, measured slower: the hardware dispatcher
// keeps more tiles in flight than a fixed grid does.)  Tile index =
// blockIdx.y * gridDim.x + blockIdx.x: a grid holds fewer than 2^32 threads
// per dimension, so launches of more tiles use rows of workgroups.
// STREAM: non-temporal loads and stores (TileArgs::io bit 3: whole lines).
template <typename R, int LOG_NT, int LOG_R, bool STREAM>
__global__ __launch_bounds__(1 << LOG_NT) void k_tile(TileArgs a)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const uint64_t t = (uint64_t)blockIdx.y * gridDim.x + blockIdx.x;
    TileKernel<R, LOG_NT, LOG_R, true, STREAM>::template run_range<false, true>(a, lds_raw, t, t + 1, 1, {nullptr, 0});
}

// The same pass with the ZB read-out of every tile into zparts.
template <typename R, int LOG_NT, int LOG_R, bool STREAM>
__global__ __launch_bounds__(1 << LOG_NT) void k_tile_z(TileArgs a, double *zparts)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const uint64_t t = (uint64_t)blockIdx.y * gridDim.x + blockIdx.x;
    // value v of tile t at zparts[v * (tiles of the launch) + t]
    TileKernel<R, LOG_NT, LOG_R, true, STREAM>::template run_range<false, true, true>(
        a, lds_raw, t, t + 1, 1, {nullptr, 0}, zparts, (uint64_t)gridDim.x * gridDim.y);
}

template <typename R, int LOG_NT, int LOG_R, bool STREAM, bool ZB>
void launch_tile_kernel(const TileArgs &a, uint64_t n_tiles, double *zparts, hipStream_t st)
{
    constexpr size_t bytes = TileKernel<R, LOG_NT, LOG_R>::LDS_BYTES;
    const void *fn = ZB ? reinterpret_cast<const void *>(&k_tile_z<R, LOG_NT, LOG_R, STREAM>)
                        : reinterpret_cast<const void *>(&k_tile<R, LOG_NT, LOG_R, STREAM>);
    // once per process (a thread-safe static initialisation); a failure
    // throws, and the next launch tries again
    static const bool ready = [fn] {
        check_no_static_lds(fn, "tile kernel");
        // launches above the default dynamic LDS limit need the attribute first
        if (bytes > 65536) {
            hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
            if (e != hipSuccess)
                fail(QS_ERR_HIP, std::string("tile kernel attribute: ") + hipGetErrorString(e));
        }
        return true;
    }();
    (void)ready;
    if (n_tiles == 0)
        return;
    // at most 2^31 threads per grid row; tile counts are powers of two
    const uint64_t row = std::min<uint64_t>(n_tiles, (1ull << 31) >> LOG_NT);
    if (n_tiles % row != 0 || n_tiles / row > 0xffffull)
        fail(QS_ERR_UNSUPPORTED, "tile count does not fit one launch");
    if constexpr (ZB)
        hipLaunchKernelGGL((k_tile_z<R, LOG_NT, LOG_R, STREAM>), dim3((unsigned)row, (unsigned)(n_tiles / row)),
                           dim3(1 << LOG_NT), bytes, st, a, zparts);
    else
        hipLaunchKernelGGL((k_tile<R, LOG_NT, LOG_R, STREAM>), dim3((unsigned)row, (unsigned)(n_tiles / row)),
                           dim3(1 << LOG_NT), bytes, st, a);
    check_launch("tile pass");
}

// MODE 0: plain loads and stores; 1: non-temporal (passes over whole 128-byte
// lines, TileArgs::io bit 3); 2: non-temporal with the per-tile read-out.
// Each mode is instantiated in a translation unit of its own, so that the
// three sets compile in parallel.
template <typename R, int LOG_NT, int LOG_R, int MODE>
void launch_tile_inst(const TileArgs &a, uint64_t n_tiles, double *zparts, hipStream_t st)
{
    if (MODE != 0 && !(a.io & 8u))
        fail(QS_ERR_UNSUPPORTED, "non-temporal tile pass over partial lines");
    launch_tile_kernel<R, LOG_NT, LOG_R, MODE != 0, MODE == 2>(a, n_tiles, zparts, st);
}

// Dispatch over the instantiated shapes: 2^6..2^10 threads, 2..32 amplitudes
// per thread, at most 128 KiB of LDS (half the tile).
template <typename R, int MODE>
void launch_tile_t(const TileArgs &a, uint64_t n_tiles, int log_r, int log_nt, double *zparts, hipStream_t st)
{
#define QS_TILE_CASE(NTB, RB)                                            \
    if (log_nt == NTB && log_r == RB) {                                  \
        if constexpr (TileKernel<R, NTB, RB>::LDS_BYTES <= 131072) {      \
            launch_tile_inst<R, NTB, RB, MODE>(a, n_tiles, zparts, st);  \
            return;                                                      \
        }                                                                \
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
