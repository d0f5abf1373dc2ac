// The interface of the fused tile kernel: the operation records it reads and
// its kernel arguments.  Kept apart from the host declarations, so that the
// stored hardware-counter measurements of the kernel are tied to the files
// that define it (the kernel sources and this one).
#pragma once

#include <cstddef>
#include <cstdint>

namespace qsim {

enum TileOpKind : int32_t {
    OP_U = 0,      // dense 2x2 on register slot `slot`
    OP_X = 1,      // exchange the pair on register slot `slot`
    OP_DIAG = 2,   // multiply by d0 (m[0..1]) / d1 (m[2..3]) selected by the target bit
    OP_NEG = 3,    // negate where every control bit is 1
    OP_REMAP = 4,  // move amplitudes through LDS to a new register layout: rmask and hbit
                   // give its register and thread tile bits, the first words of m the
                   // LDS slot (lds_swizzle) of each register slot bit (word s: slot bit s);
                   // aux & REMAP_WAVE_LOCAL: the tile bits on the wavefront-index bits of
                   // the thread id stay, so no barrier is needed
    OP_SHEAR = 5,  // on the pair (x, y) of register slot `slot`: x += p y, then y += q x, with
                   // p = (m[0], m[1]) and q = (m[2], m[3]); tlane != 0: exchange x and y
                   // first (a relabelling); no controls
    OP_PHASE = 6,  // multiply where the bit of register slot `slot` is 1 by (m[0], m[1]); no
                   // controls
    OP_SHEAR2 = 7, // two OP_SHEARs on different register slots in one record: the first on
                   // `slot` (m[0..3], exchange flag tlane), the second on slot aux & 255
                   // (m[4..7], exchange flag aux >> 8)
    OP_LSWAP = 8,  // exchange register slot bit `slot` with lane bit tlane (4 or 5) of the
                   // wavefront, in registers: the tile bit lmask (on the lane bit) moves into
                   // the slot, the tile bit rmask (on the slot) onto the lane bit; the first
                   // word of m is the slot's new LDS slot (lds_swizzle of lmask)
    OP_LANE = 9,   // dense 2x2 (m[0..7]) on thread-id bit tlane (< 4) of the layout, through
                   // lane exchanges (DPP) instead of a re-layout; no controls
};

constexpr uint32_t REMAP_WAVE_LOCAL = 1u;
constexpr uint32_t IO_BASIS = 16u;

// One operation of a fused tile pass (104 bytes, every field at least 32 bits
// wide and naturally aligned so that the kernel reads it with scalar loads).  Its controls are split by
// where the control bit lives under the register layout in force when the
// operation runs: register slots (rmask, a mask over slots), thread bits
// (lmask, a mask over tile-local index bits) and positions outside the tile
// (hmask, a mask over physical positions).  The operation acts where every
// control bit is 1.
struct TileOp {
    int32_t kind;
    int32_t slot;      // OP_U/OP_X: target register slot.  OP_DIAG: target
                       // register slot, or -1 (target is the thread bit tlane)
                       // or -2 (target outside the tile, at hbit)
    uint32_t rmask;    // OP_REMAP: register tile bits, 4 bits each (slot s at bits 4s..4s+3)
    uint32_t lmask;
    uint32_t tlane;
    uint32_t aux;      // OP_SHEAR2: the second shear's slot and exchange flag; OP_REMAP: flags
    uint64_t hmask;
    uint64_t hbit;     // OP_DIAG target outside the tile; OP_REMAP: the tile bit of each
                       // thread-id bit, 4 bits each (thread bit i at bits 4i..4i+3)
    double m[8];
};
static_assert(sizeof(TileOp) == 104, "TileOp layout");

// LDS element slot of tile-local index i in a tile of 2^k amplitudes: i with
// each higher group of 5 bits XORed into its low 5 bits.  The map is linear
// over GF(2) and invertible, so a layout's LDS slots are XORs of a per-thread
// and per-register-slot parts, and lanes whose indices differ only in high
// bits land in different banks.
constexpr uint32_t lds_swizzle(uint32_t i, int k)
{
    uint32_t r = i;
    for (int s = 5; s < k; s += 5)
        r ^= (i >> s) & 31u;
    return r;
}

// Kernel arguments of one tile pass, passed by value.  The load and store
// layouts give, for each thread-id bit and each register-slot bit, the
// physical position it addresses.
struct TileArgs {
    void *state;
    const TileOp *ops;
    int32_t n_ops;
    int32_t n_hi;                 // positions outside the tile
    uint8_t pos[16];              // tile bit b -> physical position (ascending)
    uint8_t ld_lane[16];          // load layout: thread-id bit -> position
    uint8_t ld_reg[8];            // load layout: slot bit -> position
    uint8_t st_lane[16];          // store layout: thread-id bit -> position
    uint8_t st_reg[8];            // store layout: slot bit -> position
    uint32_t io;                  // bit 0: the load layout is that of ops[0] (an OP_REMAP, then
                                  // skipped), else tile-local index j * NT + tid;
                                  // bit 1: the store layout is that of the last OP_REMAP, else
                                  // tile-local index j * NT + tid reached through LDS;
                                  // bit 2 (only with no ops): the amplitude at tile-local index
                                  // t is stored at index sperm(t) (a bit permutation);
                                  // bit 3: the lowest tile positions are the lowest
                                  // physical positions, so every load and store moves
                                  // whole 128-byte lines (non-temporal access pays);
                                  // bit 4 (IO_BASIS): nothing is read, the tiles start as
                                  // the basis state |0...0> (1 at physical index 0)
    int32_t pad;
    uint8_t sperm[16];            // tile bit b moves to tile bit sperm[b] (io bit 2)
};
static_assert(sizeof(TileArgs) == 112, "TileArgs layout");

}  // namespace qsim
