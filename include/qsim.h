/*
 * qsim.h: C boundary of the MI355X state-vector simulator.
 *
 * The operations follow the problem statement of Guerreschi, "Fast simulation
 * of quantum algorithms using circuit optimization" (arXiv:2010.09746):
 *   - a state of n qubits is the vector of its 2^n complex amplitudes
 *     (Section 2);
 *   - qubit q is bit q of the logical basis index, i = sum_q i_q 2^q, and under
 *     a qubit placement sigma the amplitude a_i is stored at physical index
 *     j(i, sigma) = sum_q i_q 2^sigma(q) (Section 2);
 *   - gates are one-qubit gates and controlled one-qubit gates, which update
 *     amplitudes in pairs (Section 2);
 *   - PermuteQubits(sigma') re-orders the stored amplitudes to a new placement
 *     (Section 2, Appendix A);
 *   - a compiled circuit is a list of ApplyGate and PermuteQubits
 *     instructions produced by the pass of Section 3 (Algorithm 1).
 *
 * Conventions for every entry point:
 *   - Every call returns a qs_status; no C++ exception crosses this boundary.
 *     On failure qs_last_error() returns a message for the calling thread.
 *   - "device" pointers are HIP device addresses on the current device;
 *     "host" pointers are ordinary CPU memory owned by the caller.
 *   - Calls that apply gates or move data are enqueued on the state's HIP
 *     stream and return before the work finishes.  Read-out calls wait for
 *     the state's stream and fill caller-owned host arrays.
 *   - A handle is not thread-safe; distinct handles are independent.
 *   - The library never frees memory it did not allocate.
 */
#ifndef QSIM_H
#define QSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qs_state qs_state;
typedef struct qs_program qs_program;
typedef struct qs_batch qs_batch;
typedef struct qs_server qs_server;

typedef enum {
    QS_C64 = 0,  /* complex64: float re, im (8 bytes per amplitude)  */
    QS_C128 = 1  /* complex128: double re, im (16 bytes per amplitude) */
} qs_dtype;

typedef enum {
    QS_OK = 0,
    QS_ERR_ARG = -1,         /* invalid argument (qubit range, sigma not a permutation, sizes) */
    QS_ERR_OOM = -2,         /* device allocation failed */
    QS_ERR_BUDGET = -3,      /* a request does not fit the memory budget */
    QS_ERR_HIP = -4,         /* a HIP runtime call or kernel launch failed */
    QS_ERR_UNSUPPORTED = -5, /* valid request outside what the library implements */
    QS_ERR_STATE = -6        /* handle in the wrong state (e.g. program compiled for another placement) */
} qs_status;

/* Gate kinds (paper, Section 2: one-qubit gates and controlled one-qubit gates). */
typedef enum {
    QS_GATE_U = 0,  /* 2x2 matrix u on qubit q0 */
    QS_GATE_CX = 1, /* controlled X: control q0, target q1 (u ignored) */
    QS_GATE_CZ = 2, /* controlled Z on q0, q1 (symmetric; u ignored) */
    QS_GATE_CU = 3  /* controlled u: control q0, target q1 */
} qs_gate_kind;

/* One gate, 80 bytes.  u holds the 2x2 matrix row-major as interleaved
 * (re, im): u00, u01, u10, u11.  Qubits are logical indices in [0, n). */
typedef struct {
    int32_t kind;
    int32_t q0;
    int32_t q1; /* -1 for one-qubit gates */
    int32_t reserved;
    double u[8];
} qs_gate;

enum { QS_FORM_PLAIN = 0, QS_FORM_PASS = 1 };
enum { QS_PERM_MOVE = 0, QS_PERM_RELABEL = 1 };

/* Options of qs_compile / qs_run_circuit.
 *   form       QS_FORM_PLAIN: one kernel launch per gate.
 *              QS_FORM_PASS: the pass of Section 3 with m = k_tile local
 *              (in-tile) qubits; each run of local gates becomes one fused tile
 *              pass over HBM.
 *   k_tile     tile qubits (at most n).  A tile is 2^k_tile amplitudes held
 *              by one workgroup; tile passes need 7 <= k_tile and a tile of at
 *              most 256 KiB (k_tile <= 14 for complex128, 15 for complex64),
 *              else the local gates run one launch each.
 *   max_swaps  r >= 1: local/global exchanges chained into one PermuteQubits.
 *              r = 1 with pinned = 0 is Algorithm 1 as printed.  r = 0: no
 *              PermuteQubits at all; runs of gates on the first k_tile
 *              positions are fused and every other gate is one launch (the
 *              fusion without the pass, for comparison).
 *   pinned     qubits at positions < pinned are never exchanged out.
 *   perm_exec  QS_PERM_MOVE: each PermuteQubits moves the amplitudes (in place)
 *              and tiles are contiguous.  QS_PERM_RELABEL: no data moves; each
 *              tile pass gathers the positions of the current local qubits.
 *   max_fuse   upper bound on gates per tile pass (0 = none).
 *   reg_bits   amplitudes per thread = 2^reg_bits inside the tile kernel
 *              (0 = chosen by the library).
 *   flags      QS_OPT_FULL_MATRICES: every one-qubit gate of a tile pass is
 *              applied as its whole 2x2 matrix.  Without it (0, the
 *              default) an uncontrolled gate M on qubit q (with q's pending
 *              factor absorbed) is factored as F [[1, 0], [q, 1]] [[1, p],
 *              [0, 1]] (or the same for M X, after an exchange that
 *              relabels register slots): two in-place shears, 8 real
 *              multiply-adds per amplitude pair instead of 16.  The left
 *              factor F is kept pending on q and absorbed by q's next
 *              one-qubit gate: F = a I + b X when q's operations up to that
 *              gate are all CNOT targets (it commutes with them; complex128
 *              only, since such factors amplify rounding errors), else
 *              M00 diag(1, z), applied before an operation that acts on q
 *              non-diagonally, with M00 in one scalar that the next gate
 *              applied whole takes.  The last gate of each qubit is applied
 *              whole.  Same result up to rounding.
 *              QS_OPT_LANE_GATES / QS_OPT_LANE_GATES_WIDE: an uncontrolled
 *              one-qubit gate whose target is on thread-id bit 0 or 1 (bits
 *              0..3 with _WIDE) of the tile layout in force may run there,
 *              applied whole through lane exchanges (DPP moves) instead of
 *              after a register re-layout through LDS: only when every ready
 *              gate that waits for a re-layout can (the re-layout is put
 *              off), or, with QS_OPT_LANE_EAGER as well, whenever it is
 *              ready.  Off by default: on the 30-qubit layered workload they
 *              cost more than the re-layouts they save.  Same result up to
 *              rounding.
 *              QS_OPT_FROM_ZERO: the run starts from |0...0> whatever the
 *              state holds (its placement still has to be the starting
 *              one).  When the first launch is a tile pass it generates the
 *              basis state in registers instead of reading the state (no
 *              preparation pass over HBM); otherwise the state is set to
 *              |0...0> first.  For qs_compile the flag is kept with the
 *              program and applies to every qs_run_program of it.
 *              QS_OPT_X_FACTORS: complex64 states keep a I + b X pending
 *              factors too (complex128 always does): no phase operations
 *              before CNOT targets, at the price of larger rounding errors
 *              (measured on a 24-qubit layered circuit against the oracle:
 *              maximum amplitude error 3.2e-8 instead of 8.8e-10, fidelity
 *              loss 9.6e-10 instead of 8.3e-13; complex64 passes 9% faster
 *              on the 32-qubit workload).
 */
enum {
    QS_OPT_FULL_MATRICES = 1,
    QS_OPT_LANE_GATES = 2,
    QS_OPT_LANE_GATES_WIDE = 4,
    QS_OPT_LANE_EAGER = 8,
    QS_OPT_FROM_ZERO = 16,
    QS_OPT_X_FACTORS = 32
};
typedef struct {
    int32_t form;
    int32_t k_tile;
    int32_t max_swaps;
    int32_t pinned;
    int32_t perm_exec;
    int32_t max_fuse;
    int32_t reg_bits;
    int32_t flags;
} qs_run_opts;

typedef struct {
    int64_t n_gates;        /* gates in the circuit */
    int64_t n_apply;        /* ApplyGate instructions on local qubits */
    int64_t n_perm;         /* PermuteQubits instructions */
    int64_t n_global;       /* gates applied while not local (Algorithm 1 fallback) */
    int64_t n_swaps;        /* local/global exchanges summed over all PermuteQubits */
    int64_t n_tile_passes;  /* fused tile kernel launches */
    int64_t n_move_passes;  /* data-movement launches for PermuteQubits */
    int64_t n_plain;        /* one-gate kernel launches */
    int64_t n_remaps;       /* register/LDS re-layouts inside all tile passes */
    double compile_ms;      /* host time of qs_compile */
} qs_program_stats;

/* Message describing the last failure on this thread ("" if none). */
const char *qs_last_error(void);

/* Properties of the current HIP device.  name: host buffer of name_len bytes. */
qs_status qs_device_info(int *cu_count, int *lds_bytes_per_cu, size_t *hbm_bytes, char *name,
                         int name_len);

/* ---- state ------------------------------------------------------------- */

/* Create an n-qubit state (1 <= n <= 34) of type dt on the current device.
 * device_buf: caller-owned device buffer of at least 2^n * (8 or 16) bytes
 *   (buf_bytes), e.g. a torch tensor; NULL lets the library allocate (and
 *   later free) it.  stream: hipStream_t for all work on this state (NULL =
 *   the default stream).  The amplitudes are set to |0...0> with the identity
 *   placement.  Also allocates a small read-out workspace. */
qs_status qs_state_create(int n, qs_dtype dt, void *device_buf, size_t buf_bytes, void *stream,
                          qs_state **out);
qs_status qs_state_destroy(qs_state *s);
qs_status qs_state_set_stream(qs_state *s, void *stream);
/* n, dtype, device buffer of the state (any pointer may be NULL). */
qs_status qs_state_info(const qs_state *s, int *n, int *dtype, void **device_buf);

/* State preparation (Section 2): |x> for logical index x, identity placement. */
qs_status qs_state_set_basis(qs_state *s, uint64_t logical_index);

/* Current placement: sigma[q] = position of qubit q (host array of n ints). */
qs_status qs_get_permutation(const qs_state *s, int *sigma);

/* ---- gates and data movement -------------------------------------------- */

/* Apply one gate (logical qubits, mapped through the placement) as one
 * kernel launch: the plain gate-by-gate form. */
qs_status qs_apply_gate(qs_state *s, const qs_gate *g);
qs_status qs_apply_gates(qs_state *s, const qs_gate *g, int64_t n_gates);

/* PermuteQubits(sigma_new) (Section 2, Appendix A): move every amplitude from
 * j(i, sigma) to j(i, sigma_new) in place.  sigma_new: host array of n ints,
 * a permutation of 0..n-1.  Bit-exact data movement. */
qs_status qs_permute_qubits(qs_state *s, const int *sigma_new);

/* ---- compiled circuits (Section 3, Algorithm 1) ------------------------- */

/* Compile n_gates gates (host array) for n qubits and amplitude type dt.
 * sigma0: host array of the placement the program will start from (NULL =
 * identity).  Host-only; device tables are uploaded on first run. */
qs_status qs_compile(const qs_gate *gates, int64_t n_gates, int n, qs_dtype dt,
                     const int *sigma0, const qs_run_opts *opts, qs_program **out);

/* Measured costs for the pass's own choices (paper, Section 3, closing
 * remark: a pass may use the simulator's benchmarks instead of the step
 * function local / global).  All in one time unit, for the state size being
 * compiled for (bench-measured, e.g. by paper_2010_09746_amd.costmodel):
 *   tile_pass   fixed cost of one fused tile pass (every amplitude read and
 *               written once)
 *   in_pass[c]  cost of one gate inside a tile pass: c = 0 a non-diagonal
 *               one-qubit gate, 1 a two-qubit gate with a non-diagonal target
 *               (CX, CU), 2 a diagonal gate (CZ, controlled or one-qubit
 *               diagonal)
 *   move        cost of moving every amplitude once (QS_PERM_MOVE: a
 *               PermuteQubits of P exchanged position pairs moves the fraction
 *               1 - 2^-P); 0 with relabelled placements
 *   plain[k]    one gate of kind k (QS_GATE_U, CX, CZ, CU) as a launch of its
 *               own (the paper's communicating gate) */
typedef struct {
    double tile_pass;
    double in_pass[3];
    double move;
    double plain[4];
} qs_pass_costs;

/* qs_compile with the pass deciding by predicted time (form QS_FORM_PASS,
 * max_swaps >= 1).  Where Algorithm 1 takes the whole chain of exchanges that
 * raise its count, and falls back to one communicating gate only when no
 * exchange helps, this pass predicts, at each PermuteQubits, the time per
 * gate of every prefix of that chain (the permutation's data movement, the
 * tile pass and its gates) and of running the first ready gate as a launch
 * of its own, and takes the cheapest; ties keep Algorithm 1's choice.  With
 * no movement or in-pass costs and plain launches costlier than a tile pass
 * it emits exactly qs_compile's instructions.  costs: host, read during the call; negative or non-finite
 * entries give QS_ERR_ARG.  Otherwise as qs_compile. */
qs_status qs_compile_costed(const qs_gate *gates, int64_t n_gates, int n, qs_dtype dt, const int *sigma0,
                            const qs_run_opts *opts, const qs_pass_costs *costs, qs_program **out);
qs_status qs_program_destroy(qs_program *p);
qs_status qs_program_get_stats(const qs_program *p, qs_program_stats *out);
/* Work of a compiled program by class, for a cost model that prices each
 * class with measured device costs (paper, Section 3: a pass may use the
 * simulator's own benchmarks instead of the local/global step function).
 * out[c] (host, cap doubles, c < QS_OPC_COUNT) receives, per class:
 *   QS_OPC_TILE_PASS   tile-kernel launches
 *   QS_OPC_U .. QS_OPC_REMAP  operations inside tile passes, each weighted by
 *                      the fraction of tiles that execute it (2^-h for h
 *                      control positions outside the tile)
 *   QS_OPC_DISPATCH    fetched operations that move no data on a tile: uniform
 *                      exchanges (relabels) and skipped conditional operations
 *   QS_OPC_PLAIN_*     one-gate launches by gate kind
 *   QS_OPC_MOVE        data-movement launches, QS_OPC_MOVE_FRACTION the sum
 *                      of the fractions of amplitudes they move
 *   QS_OPC_SHEAR       one-qubit updates as two shears (see flags)
 *   QS_OPC_PHASE       pending diagonals applied on their own (see flags)
 *   QS_OPC_LSWAP       exchanges of a register bit with a lane bit in registers
 *   QS_OPC_LANE        one-qubit gates through lane exchanges (see flags)
 *   QS_OPC_REMAP_WAVE  re-layouts that keep the tile bits on the wavefront
 *                      bits of the thread id (no barrier; also in QS_OPC_REMAP)
 * Writes min(cap, QS_OPC_COUNT) entries. */
enum {
    QS_OPC_TILE_PASS = 0,
    QS_OPC_U = 1,          /* one-qubit 2x2 without in-tile controls */
    QS_OPC_U_CTRL = 2,     /* controlled 2x2 with in-tile controls */
    QS_OPC_X_REG = 3,      /* exchange controlled by register bits */
    QS_OPC_X_LANE = 4,     /* exchange controlled by thread bits */
    QS_OPC_NEG = 5,        /* CZ sign flip */
    QS_OPC_DIAG = 6,       /* diagonal one-qubit or controlled-diagonal gate */
    QS_OPC_REMAP = 7,      /* register re-layout through LDS */
    QS_OPC_DISPATCH = 8,
    QS_OPC_PLAIN_U = 9,
    QS_OPC_PLAIN_CU = 10,
    QS_OPC_PLAIN_CX = 11,
    QS_OPC_PLAIN_CZ = 12,
    QS_OPC_MOVE = 13,
    QS_OPC_MOVE_FRACTION = 14,
    QS_OPC_SHEAR = 15,     /* one-qubit update as two shears */
    QS_OPC_PHASE = 16,     /* pending diagonal applied on its own */
    QS_OPC_LSWAP = 17,     /* register slot bit <-> lane bit exchange (no LDS) */
    QS_OPC_LANE = 18,      /* one-qubit 2x2 on a lane bit through lane exchanges */
    QS_OPC_REMAP_WAVE = 19, /* re-layouts (counted in QS_OPC_REMAP too) local to each wavefront: no barrier */
    QS_OPC_COUNT = 20
};
qs_status qs_program_op_counts(const qs_program *p, double *out, int cap);

/* Instruction list of the pass as int32 words: 0 v = ApplyGate(v) local;
 * 1 s_0..s_{n-1} = PermuteQubits(s); 2 v = ApplyGate(v) not local.
 * Writes up to cap words into buf (host) and the full length into *len. */
qs_status qs_program_instructions(const qs_program *p, int32_t *buf, int64_t cap, int64_t *len);

/* Enqueue a compiled program on the state's stream.  The state's placement
 * must equal the program's sigma0; afterwards it is the program's final one. */
qs_status qs_run_program(qs_state *s, const qs_program *p);
/* Compile with the state's placement and run (Section 3).  In the pass form
 * each segment is enqueued as soon as the pass has fixed the permutation that
 * follows it, so the device starts while the host is still compiling.  Returns
 * after the state's stream is synchronised.  Gates are checked before any
 * launch; an error after launches were enqueued (a HIP failure) leaves the
 * state with a partly applied circuit.  opts NULL: the pass form, k_tile 12,
 * r = 1, moved placements. */
qs_status qs_run_circuit(qs_state *s, const qs_gate *gates, int64_t n_gates,
                         const qs_run_opts *opts);

/* qs_run_circuit with the pass deciding by predicted time, as
 * qs_compile_costed (costs: host, read during the call).  The placement
 * choices and the launches they lead to are those of qs_compile_costed;
 * each segment's tile pass is enqueued as soon as the permutation after it is
 * chosen. */
qs_status qs_run_circuit_costed(qs_state *s, const qs_gate *gates, int64_t n_gates, const qs_run_opts *opts,
                                const qs_pass_costs *costs);

/* qs_run_circuit (costs NULL) or qs_run_circuit_costed, then <Z_q> of the
 * final state as qs_expect_z gives it (Section 2: measurement), with the
 * read-out folded into the last tile pass: each of its tiles also writes the
 * sum of |a|^2 and the sums over the amplitudes whose bit is 1 at each of the
 * tile's positions (FP64, fixed order), and a small kernel folds them into
 * the per-position sums, so no read-out pass over the state runs.  CNOTs and
 * CZs run on their own after that pass are allowed (a CZ changes no bit's
 * probability, a CNOT makes its target bit the XOR of two bits; at most one
 * tile bit per XOR); after any other launch, or a pass that does not move
 * whole 128-byte lines, the read-out pass of qs_expect_z runs instead.  The
 * last tile pass and the launches after it are enqueued once the program is
 * complete.  expect_z: host, n doubles (logical qubit order).  Same results
 * as qs_run_circuit followed by qs_expect_z, up to the order of the FP64
 * additions. */
qs_status qs_run_circuit_expect_z(qs_state *s, const qs_gate *gates, int64_t n_gates, const qs_run_opts *opts,
                                  const qs_pass_costs *costs, double *expect_z);

/* ---- allocation-free run -------------------------------------------------- */

/* Tile operations a program run by qs_run_program_noalloc may hold. */
#define QS_NOALLOC_MAX_OPS 32768

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the launches
 * of qs_run_program, with the program's operation table copied (on the
 * state's stream) into a fixed array of the library instead of a device
 * buffer allocated on first run.  Calls no hipMalloc, hipFree or other
 * allocating routine.  The array holds QS_NOALLOC_MAX_OPS records of 104
 * bytes (3.25 MiB); each device the library runs on keeps its own copy until
 * the process ends.  Every call on a device overwrites it: calls on one
 * stream are ordered, calls that overlap on one device (other streams or
 * threads) race.  The state's device must be the current device
 * (QS_ERR_STATE otherwise).  QS_ERR_ARG for a program with more than
 * QS_NOALLOC_MAX_OPS tile operations; the other checks and errors are those
 * of qs_run_program. */
qs_status qs_run_program_noalloc(qs_state *s, const qs_program *p);

/* ---- read-out (FP64 accumulation) --------------------------------------- */

/* Amplitudes at count logical indices (host array) into out (host, 2*count
 * doubles, interleaved re, im). */
qs_status qs_read_amplitudes(qs_state *s, const uint64_t *logical_idx, int64_t count, double *out);
/* All 2^n amplitudes in logical order into out (host, 2^(n+1) doubles). */
qs_status qs_read_state(qs_state *s, double *out);
/* <Z_q> = sum_i |a_i|^2 (1 - 2 i_q) for q = 0..n-1 into out (host, n doubles). */
qs_status qs_expect_z(qs_state *s, double *out);
/* sum_i |a_i|^2 into *out. */
qs_status qs_norm(qs_state *s, double *out);
/* Both states must have the same n.  loss = 1 - |<a|b>|^2 / (<a|a><b|b>),
 * max_abs_diff = max_i |a_i - b_i| over logical indices, all in FP64. */
qs_status qs_fidelity(qs_state *a, qs_state *b, double *loss, double *max_abs_diff);
/* Wait for all work enqueued on the state's stream. */
qs_status qs_synchronize(qs_state *s);

/* ---- batching form ---------------------------------------------------------- */

/* Options of a batch (and of a server, which uses k_tile, max_swaps, pinned,
 * reg_bits, max_fuse, wg_per_cu and chunk).
 *   k_tile     batch: largest tile; circuit c uses 2^k amplitudes per tile
 *              with k = min(n_c, k_tile) (a circuit of at most k_tile qubits
 *              is one tile: its whole state in one workgroup, all its gates in
 *              one pass), 9 <= k_tile <= 12, every n_c >= 9.  Server: the
 *              tile size of every request (7 <= k_tile <= every n).
 *   max_swaps  r of the pass (see qs_run_opts); placements are relabelled
 *   pinned     positions never exchanged out (see qs_run_opts)
 *   reg_bits   server: amplitudes per thread = 2^reg_bits (0 = library
 *              choice).  Batch: ignored (256 threads per tile,
 *              2^(k - 8) amplitudes each)
 *   max_fuse   gates per tile pass bound (0 = none)
 *   wg_per_cu  workgroups per compute unit of the persistent launch (0 = 4)
 *   chunk      tiles per work item (0 = 1)
 *   use_graph  batch: 1 = capture the run once in a HIP graph and replay it
 *   wait_ms    batch: a work item gives up waiting for its circuit's previous
 *              pass after this long (0 = 2000); the run then reports
 *              QS_ERR_HIP.  -1: every wait gives up at once (a test of that
 *              path: the launch still drains and the run reports the error) */
typedef struct {
    int32_t k_tile;
    int32_t max_swaps;
    int32_t pinned;
    int32_t reg_bits;
    int32_t max_fuse;
    int32_t wg_per_cu;
    int32_t chunk;
    int32_t use_graph;
    int32_t wait_ms;
    int32_t reserved;
} qs_batch_opts;

typedef struct {
    int64_t n_gates, n_perm, n_passes, n_tiles, n_items;
    double state_bytes, compile_ms;
} qs_batch_stats;

/* Compile count circuits (circuit c: n_qubits[c] qubits, gates[c] a host array
 * of n_gates[c] gates) for execution together.  Each circuit is compiled with
 * its own tile size (see qs_batch_opts.k_tile) and its tile passes become work
 * items (chunk tiles each).  A run is one persistent launch: workgroups take
 * items in a fixed order by ticket, and an item whose circuit's previous pass
 * is not complete waits for it (the order puts every pass's items after all
 * items of the pass before it, which guarantees progress).  The first pass of
 * each circuit starts from |0...0> without reading the state; the workgroup
 * that completes a circuit's last pass reduces its read-out.  The library
 * allocates one device buffer holding every state (complex64 or complex128),
 * the compiled tables and its own HIP stream.  Compilation runs on host
 * threads. */
qs_status qs_batch_create(int count, const int *n_qubits, const qs_gate *const *gates, const int64_t *n_gates,
                          qs_dtype dt, const qs_batch_opts *opts, qs_batch **out);
/* Enqueue one run: a small kernel that clears the run's counters, then the
 * persistent launch.  With use_graph both are captured in a HIP graph on the
 * first call and replayed after. */
qs_status qs_batch_run(qs_batch *b);
/* Wait for the last run; z0[c] = <Z_0> and norms[c] = sum |a|^2 of circuit c
 * (host arrays of count doubles, FP64 accumulation; either may be NULL).  The
 * wait is bounded: a run that has not finished after 60 s plus four times
 * wait_ms gets its waits aborted from the host and QS_ERR_HIP is returned, as
 * it is when a work item gave up waiting. */
qs_status qs_batch_results(qs_batch *b, double *z0, double *norms);
/* Amplitudes of one circuit (n <= 26) in logical order into out (host,
 * 2^(n+1) doubles); waits for the last run as qs_batch_results does. */
qs_status qs_batch_read_state(qs_batch *b, int circuit, double *out);
qs_status qs_batch_get_stats(const qs_batch *b, qs_batch_stats *out);
qs_status qs_batch_synchronize(qs_batch *b);
qs_status qs_batch_destroy(qs_batch *b);

/* The host-side plan of a batch, without a device: the pass table (circuit by
 * circuit) and the work items in ticket order, as qs_batch_create builds
 * them.  Item i covers tiles [t0, t1) of pass `pass` and may start once pass
 * `dep` (-1: none) has completed `need` tiles.  Writes up to pass_cap and
 * item_cap records (host arrays) and the full counts. */
typedef struct {
    int32_t circuit, level, k_tile, last;
    int64_t tiles;
} qs_batch_pass_info;
typedef struct {
    int32_t pass, dep;
    int64_t t0, t1, need;
} qs_batch_item_info;
qs_status qs_batch_plan(int count, const int *n_qubits, const qs_gate *const *gates, const int64_t *n_gates,
                        qs_dtype dt, const qs_batch_opts *opts, qs_batch_pass_info *passes, int64_t pass_cap,
                        int64_t *n_passes, qs_batch_item_info *items, int64_t item_cap, int64_t *n_items);

/* ---- serving form ------------------------------------------------------------ */

/* A server keeps admitted requests' states resident and advances them by
 * continuous batching: every step runs the next tile pass of every resident
 * request (one shared launch, plus a launch of its own for each request large
 * enough to fill the device; see qs_server_set_solo_tiles); requests join at
 * step boundaries and leave when their last pass has run and their read-out
 * is copied to the host.
 *   dt, opts     amplitude type and pass options shared by all requests
 *                (opts->use_graph is ignored)
 *   hbm_budget   bytes of request states that may be resident at once
 *   max_slots    resident requests at once (1..4096)
 *   max_samples  sampled amplitudes per request (read-out)
 * The server allocates its own stream, a device arena for pass tables, tile
 * operations and read-outs, and pinned host buffers for results. */
qs_status qs_server_create(qs_dtype dt, const qs_batch_opts *opts, size_t hbm_budget, int max_slots,
                           int max_samples, qs_server **out);
/* Requests whose passes have at least min_tiles tiles (2^(n - k_tile)) run
 * each pass as a tile-pass launch of their own inside the step (one workgroup
 * per tile, as qs_run_program does), after the shared launch of the smaller
 * requests; 0: every pass goes into the shared launch.  Default 2^10 tiles
 * (a pass of that many tiles fills the device by itself).
 * Results do not depend on it.  QS_ERR_ARG for min_tiles < 0, QS_ERR_STATE
 * while a step is in flight. */
qs_status qs_server_set_solo_tiles(qs_server *s, int64_t min_tiles);
qs_status qs_server_destroy(qs_server *s);
/* 1 in *fits if a state of n qubits can be admitted now (budget and slots). */
qs_status qs_server_fits(const qs_server *s, int n, int *fits);
/* Admit a compiled program (compiled for this server's dt with
 * QS_PERM_RELABEL, k_tile = opts->k_tile, identity start placement).
 * state_buf: caller-owned device buffer of 2^n amplitudes (not freed by the
 * server; it must stay valid until qs_server_release).  samples: count
 * logical basis indices (host) whose amplitudes are returned.  Fails with
 * QS_ERR_BUDGET when the budget or the slots are exhausted. */
qs_status qs_server_admit(qs_server *s, const qs_program *p, void *state_buf, size_t buf_bytes,
                          const uint64_t *samples, int count, int64_t *request_id);
/* Enqueue one step; *n_running receives the requests advanced.  Up to two
 * steps may be in flight: the next step can be enqueued before the previous
 * one is waited for (QS_ERR_STATE with two pending).  Requests admitted
 * between two launches join the later one.  Large requests' passes run on
 * up to three side streams forked from and joined back into the server's
 * stream, concurrently with the step's shared launch. */
qs_status qs_server_step_launch(qs_server *s, int *n_running);
/* Wait for the oldest step in flight; writes the ids of requests that
 * completed in it (up to cap) into ids and their number into *n_done. */
qs_status qs_server_step_wait(qs_server *s, int64_t *ids, int cap, int *n_done);
/* Results of a completed request: z (host, n doubles) = <Z_q>, amps (host,
 * 2*count doubles, interleaved re, im) and *norm, all accumulated in FP64. */
qs_status qs_server_result(qs_server *s, int64_t request_id, double *z, double *amps, double *norm);
/* Forget a completed request (its state buffer may then be reused). */
qs_status qs_server_release(qs_server *s, int64_t request_id);

/* ---- measurement ---------------------------------------------------------- */

/* Per kernel class: launches recorded, summed device time between HIP events
 * recorded on the launching stream around each launch, and the algorithmic
 * HBM bytes of those launches (every amplitude a launch must read and write,
 * counted once). */
typedef struct {
    char name[32];
    int64_t launches;
    double total_ms;
    double bytes;
} qs_profile_entry;

/* on != 0: record events around every subsequent launch (all states, this
 * process); 0: stop recording. */
qs_status qs_profile_enable(int on);
/* Wait for the recorded events, write up to cap entries (host array) and the
 * number of classes into *n_out, and clear the records. */
qs_status qs_profile_read(qs_profile_entry *out, int cap, int *n_out);

#ifdef __cplusplus
}
#endif

#endif /* QSIM_H */
