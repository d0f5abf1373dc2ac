// Internal declarations shared by the host runtime, the compiler and the HIP
// kernels of the simulator library.  Not part of the public boundary
// (include/qsim.h).
#pragma once

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "qsim.h"
#include "tile_args.h"

namespace qsim {

// ---------------------------------------------------------------------------
// gate analysis

// How a gate acts on one of its qubits.
enum Act : int { ACT_NONE = 0, ACT_Z = 1, ACT_X = 2, ACT_G = 3 };

struct GateInfo {
    int kind, q0, q1;
    int act0, act1;   // action on q0 / q1
    int nq;           // 1 or 2
    int target;       // qubit acted on non-diagonally, -1 if the gate is diagonal
    const double *u;  // matrix of the source record
};

int matrix_action(const double *u);
GateInfo analyse(const qs_gate &g);
bool gates_commute(const qs_gate &a, const GateInfo &ia, const qs_gate &b, const GateInfo &ib);

constexpr int MAX_TILE_BITS = 15;
constexpr int MIN_TILE_BITS = 7;
constexpr int MAX_QUBITS = 34;          // states
constexpr int MAX_COMPILE_QUBITS = 63;  // host-only compilation
constexpr size_t MAX_TILE_BYTES = 262144;   // one tile of a pass (LDS holds half of it)
constexpr size_t MAX_BATCH_TILE_BYTES = 131072;  // one tile of the batching and serving forms
constexpr int DIRECT_RUN_BYTES = 128;       // contiguous bytes a direct tile load or store keeps together


// ---------------------------------------------------------------------------
// batching form: one persistent launch over many circuits

// One tile pass of one circuit of a batch (device memory).
struct BatchPass {
    TileArgs t;       // the circuit's state, this pass's ops and tile positions
    uint32_t ntiles;  // tiles of this pass = 2^(n - k)
    int32_t last;     // 1: write read-out partials after the pass
    int32_t zpos;     // physical position of qubit 0
    int32_t circuit;  // index of the pass's circuit
    uint64_t part;    // first read-out partial (two doubles per tile) of the circuit
};

// Single-launch batch executor.  Work item: tiles [t0, t1) of pass `pass`,
// whose tile has 2^(8 + shape) amplitudes (256 threads x 2^shape).  It may
// start once pass `dep` (the circuit's previous pass; -1: none) has completed
// `need` tiles (all of them).  Items are listed in an order in which every
// dependency precedes its dependents.
struct QueueItem {
    uint32_t pass, t0, t1;
    int32_t dep;
    uint32_t need, shape, pad0, pad1;
};
struct QueueArgs {
    const BatchPass *passes;
    const QueueItem *items;
    uint32_t n_items, n_circuits;
    uint32_t *next;            // device: the next ticket (zero before a run)
    uint32_t *done;            // device: tiles completed per pass (zero before a run)
    uint32_t *flags;           // host-pinned: [0] abort (set by the host), [1] set by a wait that gave up
    double *partials;          // two per tile of each circuit's last pass
    double *out;               // two per circuit: <Z_0>, norm
    const uint64_t *part_off;  // per circuit: its first partial
    const uint32_t *part_cnt;  // per circuit: its number of partials (tiles of the last pass)
    uint64_t wait_ticks;       // longest wait for a dependency, in 100 MHz clock ticks
};

// A range of tiles of one pass: the unit of work of a level launch.
struct BatchItem {
    uint32_t pass, t0, t1, pad;
};

// One level: every circuit's pass of that index; the items of a level are
// independent of each other, and levels run in launch order.
struct BatchArgs {
    const BatchPass *passes;
    const BatchItem *items;
    uint32_t i0, i1;       // items of this level
    double *partials;
};

// ---------------------------------------------------------------------------
// compiled program

enum LaunchType : int { L_TILE = 0, L_PLAIN = 1, L_MOVE = 2 };

struct Launch {
    int type = L_PLAIN;
    // L_TILE
    int k = 0, log_r = 0, log_nt = 0;
    std::vector<int> pos;         // sorted tile positions
    int op_begin = 0, op_count = 0;
    uint32_t io = 0;              // TileArgs::io
    uint8_t ld_lane[16] = {}, ld_reg[8] = {}, st_lane[16] = {}, st_reg[8] = {};  // TileArgs layouts
    // L_PLAIN
    qs_gate gate{};               // qubits already mapped to physical positions
    // L_MOVE
    std::vector<int> pi;          // physical position p moves to pi[p]
};

struct Instr {
    int type;                     // 0 apply, 1 perm, 2 global
    int gate;
    std::vector<int> sigma;
};

struct PassStats {
    int64_t n_apply = 0, n_perm = 0, n_global = 0, n_swaps = 0;
};

// Pass of Section 3 (Algorithm 1) with the r / pinned extensions.
std::vector<Instr> run_pass(const qs_gate *g, int64_t ng, int n, int m, int r, int pinned,
                            const std::vector<int> &sigma0, PassStats *st);

class PassState;
struct Dag {
    std::vector<std::vector<int>> pred, succ;
};
// The same pass, one iteration per step(): the instructions of the sweep and
// the PermuteQubits (or global gate) that follows it are appended to out;
// false once every gate is scheduled.
// With costs, each PermuteQubits (or the fallback gate) is chosen by
// predicted time per gate instead (see qs_compile_costed).
class PassRunner {
public:
    PassRunner(const qs_gate *g, int64_t ng, int n, int m, int r, int pinned, const std::vector<int> &sigma0,
               const qs_pass_costs *costs = nullptr);
    ~PassRunner();
    PassRunner(const PassRunner &) = delete;
    PassRunner &operator=(const PassRunner &) = delete;
    // One half of an iteration of Algorithm 1 per call: first the ApplyGate
    // instructions of every gate that is ready and local, then the
    // PermuteQubits (or the fallback gate).  False when the circuit is done.
    bool step(std::vector<Instr> &out);
    // after the first half: the run of ApplyGate instructions just emitted is
    // complete (a PermuteQubits, a fallback gate or the end follows)
    bool run_closed() const { return swept_; }
    const PassStats &stats() const { return stats_; }
    const std::vector<GateInfo> &gate_info() const { return gi_; }

private:
    int n_, m_, r_, pinned_;
    bool costed_ = false;
    qs_pass_costs costs_{};
    std::vector<GateInfo> gi_;
    Dag dag_;
    PassState *ps_ = nullptr;
    std::vector<int> sigma_, emitted_;
    PassStats stats_;
    bool swept_ = false;
};

struct Program {
    int n = 0;
    qs_dtype dt = QS_C128;
    qs_run_opts opts{};
    std::vector<int> sigma0, sigma_final;
    std::vector<Instr> instrs;
    std::vector<Launch> launches;
    std::vector<TileOp> ops;
    qs_program_stats stats{};
    // device copy of ops (per device, uploaded on first run)
    int dev = -1;
    TileOp *d_ops = nullptr;
};

// Compile a circuit.  With progress, the pass form calls it after each pass
// iteration, once the launches of every completed segment are in p.launches
// (and their operations in p.ops); launches already there never change.
void compile_program(const qs_gate *g, int64_t ng, int n, qs_dtype dt, const int *sigma0,
                     const qs_run_opts &o, Program &p, const std::function<void(Program &)> &progress = {},
                     const qs_pass_costs *costs = nullptr);

}  // namespace qsim

// handle behind qs_program
struct qs_program {
    qsim::Program p;
};

namespace qsim {

// kernel arguments of a tile launch: op count, positions and load/store
// layouts (the state and ops pointers and n_hi are the caller's)
void tile_args_from_launch(const Launch &L, TileArgs &a);
// kernel arguments of an empty tile pass over tile positions 0..k-1, or over
// the given ascending positions
void tile_args_identity(int k, int log_nt, int log_r, TileArgs &a);
void tile_args_for_positions(const std::vector<int> &pos, int log_nt, int log_r, TileArgs &a);

// choose register bits / threads for a tile of k bits
// Tile shape: 2^log_r amplitudes per thread (reg_bits_opt, or pass_reg_bits
// when 0), clamped to 64..1024 threads.
void tile_shape(int k, qs_dtype dt, int reg_bits_opt, int *log_r, int *log_nt);
// register bits of a tile when none are asked for (measured)
int pass_reg_bits(int k, qs_dtype dt);

// ---------------------------------------------------------------------------
// state access for entry points defined outside api.cpp

// The checks of qs_run_program (qubit count, amplitude type, starting
// placement) without running anything.
void check_program_on(const qs_state *s, const Program &p);
// Enqueue every launch of p on the state's stream with the operation table
// read from d_ops (device memory holding p.ops), then take p's final
// placement.  Allocates nothing on the device.
void run_program_with_ops(qs_state *s, const Program &p, const TileOp *d_ops);
void *state_stream(const qs_state *s);  // the state's hipStream_t
int state_device(const qs_state *s);    // the device the state was created on
// f() with exceptions turned into a status and the per-thread message
qs_status guarded(const std::function<void()> &f);

// ---------------------------------------------------------------------------
// error reporting

struct Error {
    qs_status code;
    std::string msg;
};
[[noreturn]] void fail(qs_status code, const std::string &msg);
// message returned by qs_last_error() on this thread
void set_last_error(const std::string &msg);

}  // namespace qsim
