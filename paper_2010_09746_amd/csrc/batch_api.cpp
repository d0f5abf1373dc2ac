// Batching form (C boundary): many independent circuits of different sizes,
// each compiled with its own tile size, executed by one persistent launch
// that takes ranges of tiles from a ticketed work list and waits, per item,
// for the circuit's previous pass.  The launch (after a small kernel that
// clears its counters) is captured once in a HIP graph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"
#include "kernels.h"

using namespace qsim;

namespace {

// Host-only plan of a batch: compiled programs, the pass table (circuit by
// circuit) and the work items in ticket order.
struct PlanPass {
    int circuit = 0, level = 0, k = 0, last = 0;
    uint32_t tiles = 0;
    const Launch *launch = nullptr;  // NULL: the empty pass of a circuit without gates
};

struct BatchPlan {
    std::vector<Program> progs;
    std::vector<int> k;                          // tile qubits of each circuit
    std::vector<PlanPass> passes;
    std::vector<std::vector<int>> circ_passes;   // pass indices of each circuit, in order
    std::vector<QueueItem> items;
};

constexpr int BATCH_MIN_TILE = QUEUE_LOG_NT + QUEUE_MIN_SHAPE;  // 9
constexpr int BATCH_MAX_TILE = QUEUE_LOG_NT + QUEUE_MAX_SHAPE;  // 12

void check_opts(const qs_batch_opts &o)
{
    if (o.k_tile < BATCH_MIN_TILE || o.k_tile > BATCH_MAX_TILE)
        fail(QS_ERR_ARG, "k_tile of a batch must be in [9, 12]");
    if (o.max_swaps < 0 || o.pinned < 0 || o.max_fuse < 0 || o.chunk < 0 || o.wg_per_cu < 0 || o.wait_ms < -1)
        fail(QS_ERR_ARG, "negative batch option");
}

// Compile every circuit (host threads) with k = min(n, k_tile) and order the
// work: level by level (the L-th pass of every circuit), and within a level
// the circuits with the most work left first.  Every item of a circuit's
// pass L comes after every item of its pass L - 1, which the executor's
// progress argument needs.
void plan_batch(int count, const int *n, const qs_gate *const *gates, const int64_t *n_gates, qs_dtype dt,
                const qs_batch_opts &o, BatchPlan &bp)
{
    check_opts(o);
    bp.progs.assign(count, Program());
    bp.k.resize(count);
    for (int c = 0; c < count; ++c) {
        if (n[c] < BATCH_MIN_TILE || n[c] > MAX_QUBITS)
            fail(QS_ERR_ARG, "every circuit of a batch needs 9 <= n <= 34 (circuit " + std::to_string(c) + ")");
        if (n_gates[c] < 0 || (n_gates[c] > 0 && !gates[c]))
            fail(QS_ERR_ARG, "bad gate array (circuit " + std::to_string(c) + ")");
        bp.k[c] = std::min(n[c], o.k_tile);
    }
    std::vector<std::string> errs(count);
    const unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (unsigned w = 0; w < nth; ++w)
        th.emplace_back([&, w] {
            for (int c = (int)w; c < count; c += (int)nth) {
                qs_run_opts ro{};
                ro.form = QS_FORM_PASS;
                ro.k_tile = bp.k[c];
                ro.max_swaps = std::max(1, o.max_swaps);
                ro.pinned = std::min(o.pinned, bp.k[c]);
                ro.perm_exec = QS_PERM_RELABEL;
                ro.max_fuse = o.max_fuse;
                ro.reg_bits = bp.k[c] - QUEUE_LOG_NT;
                try {
                    compile_program(gates[c], n_gates[c], n[c], dt, nullptr, ro, bp.progs[c]);
                } catch (const Error &e) {
                    errs[c] = e.msg;
                }
            }
        });
    for (auto &t : th)
        t.join();
    for (int c = 0; c < count; ++c)
        if (!errs[c].empty())
            fail(QS_ERR_ARG, "circuit " + std::to_string(c) + ": " + errs[c]);

    // pass table: each circuit's tile passes; a circuit without gates gets
    // one empty pass, so that its state and read-out are still produced
    bp.passes.clear();
    bp.circ_passes.assign(count, {});
    for (int c = 0; c < count; ++c) {
        const Program &p = bp.progs[c];
        std::vector<const Launch *> tl;
        for (const Launch &L : p.launches) {
            if (L.type != L_TILE || L.k != bp.k[c] || L.log_nt != QUEUE_LOG_NT)
                fail(QS_ERR_UNSUPPORTED, "batch circuit " + std::to_string(c) + " needs a launch other than a tile pass");
            tl.push_back(&L);
        }
        const int np = std::max<int>(1, (int)tl.size());
        for (int i = 0; i < np; ++i) {
            PlanPass P;
            P.circuit = c;
            P.level = i;
            P.k = bp.k[c];
            P.last = i == np - 1;
            P.tiles = (uint32_t)(1ull << (n[c] - bp.k[c]));
            P.launch = tl.empty() ? nullptr : tl[i];
            bp.circ_passes[c].push_back((int)bp.passes.size());
            bp.passes.push_back(P);
        }
    }
    // work items: level by level; within a level, circuits by the amplitudes
    // their remaining passes touch (most first)
    const uint32_t chunk = (uint32_t)std::max(1, o.chunk);
    size_t max_np = 0;
    for (auto &v : bp.circ_passes)
        max_np = std::max(max_np, v.size());
    std::vector<std::vector<double>> left(count);
    for (int c = 0; c < count; ++c) {
        const auto &v = bp.circ_passes[c];
        left[c].assign(v.size() + 1, 0.0);
        for (int i = (int)v.size() - 1; i >= 0; --i)
            left[c][i] = left[c][i + 1] + std::ldexp(1.0, n[c]);
    }
    bp.items.clear();
    std::vector<int> order(count);
    for (size_t lvl = 0; lvl < max_np; ++lvl) {
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            const double la = lvl < bp.circ_passes[a].size() ? left[a][lvl] : -1.0;
            const double lb = lvl < bp.circ_passes[b].size() ? left[b][lvl] : -1.0;
            return la > lb;
        });
        for (int c : order) {
            if (lvl >= bp.circ_passes[c].size())
                continue;
            const int pi = bp.circ_passes[c][lvl];
            const PlanPass &P = bp.passes[pi];
            const int dep = lvl > 0 ? bp.circ_passes[c][lvl - 1] : -1;
            for (uint32_t t = 0; t < P.tiles; t += chunk) {
                QueueItem it{};
                it.pass = (uint32_t)pi;
                it.t0 = t;
                it.t1 = std::min(P.tiles, t + chunk);
                it.dep = dep;
                it.need = dep >= 0 ? bp.passes[dep].tiles : 0;
                it.shape = (uint32_t)(P.k - QUEUE_LOG_NT);
                bp.items.push_back(it);
            }
        }
    }
}

void hipchk(hipError_t e, const char *what)
{
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(e == hipErrorOutOfMemory ? QS_ERR_OOM : QS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
    }
}

template <typename F> qs_status guard(F &&f)
{
    try {
        f();
        set_last_error("");
        return QS_OK;
    } catch (const Error &e) {
        set_last_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc &) {
        set_last_error("host allocation failed");
        return QS_ERR_OOM;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return QS_ERR_ARG;
    } catch (...) {
        set_last_error("unknown error");
        return QS_ERR_ARG;
    }
}

}  // namespace

struct qs_batch {
    int count = 0;
    qs_dtype dt = QS_C64;
    qs_batch_opts opts{};
    int grid = 0;
    hipStream_t stream = nullptr;
    hipEvent_t done_ev = nullptr;
    std::vector<int> n;
    std::vector<uint64_t> start;  // element offset of each state
    uint64_t total = 0;
    std::vector<BatchPass> passes;
    std::vector<QueueItem> items;
    std::vector<uint64_t> part_off;
    std::vector<uint32_t> part_cnt;
    uint64_t n_partials = 0;
    uint64_t n_words = 0;         // ticket + per-pass counters
    // device
    void *d_state = nullptr;
    TileOp *d_ops = nullptr;
    BatchPass *d_passes = nullptr;
    QueueItem *d_items = nullptr;
    uint32_t *d_words = nullptr;
    double *d_partials = nullptr, *d_out = nullptr;
    uint64_t *d_part_off = nullptr;
    uint32_t *d_part_cnt = nullptr;
    uint32_t *h_flags = nullptr;  // host-pinned: [0] abort, [1] a wait gave up
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    qs_batch_stats stats{};
};

namespace {

template <typename T> void upload(T *&dst, const std::vector<T> &src, const char *what)
{
    hipchk(hipMalloc(&dst, std::max<size_t>(1, src.size()) * sizeof(T)), what);
    if (!src.empty())
        hipchk(hipMemcpy(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice), what);
}

void free_batch(qs_batch *b)
{
    if (b->exec)
        (void)hipGraphExecDestroy(b->exec);
    if (b->graph)
        (void)hipGraphDestroy(b->graph);
    void *ptrs[] = {b->d_state, b->d_ops, b->d_passes, b->d_items, b->d_words,
                    b->d_partials, b->d_out, b->d_part_off, b->d_part_cnt};
    for (void *p : ptrs)
        if (p)
            (void)hipFree(p);
    if (b->h_flags)
        (void)hipHostFree(b->h_flags);
    if (b->done_ev)
        (void)hipEventDestroy(b->done_ev);
    if (b->stream)
        (void)hipStreamDestroy(b->stream);
}

QueueArgs queue_args(qs_batch *b)
{
    QueueArgs q{};
    q.passes = b->d_passes;
    q.items = b->d_items;
    q.n_items = (uint32_t)b->items.size();
    q.n_circuits = (uint32_t)b->count;
    q.next = b->d_words;
    q.done = b->d_words + 4;
    q.flags = b->h_flags;
    q.partials = b->d_partials;
    q.out = b->d_out;
    q.part_off = b->d_part_off;
    q.part_cnt = b->d_part_cnt;
    const int ms = b->opts.wait_ms > 0 ? b->opts.wait_ms : b->opts.wait_ms < 0 ? 0 : 2000;
    q.wait_ticks = (uint64_t)ms * 100000ull;  // 100 MHz; 0: every wait gives up at once
    return q;
}

void enqueue(qs_batch *b)
{
    launch_queue_reset(b->d_words, b->n_words, b->stream);
    const QueueArgs q = queue_args(b);
    const int grid = (int)std::min<size_t>((size_t)b->grid, std::max<size_t>(1, b->items.size()));
    if (b->dt == QS_C64)
        launch_batch_queue_f32(q, grid, b->stream);
    else
        launch_batch_queue_f64(q, grid, b->stream);
}

// Wait for the last run, giving up after a bound: then the host sets the
// abort flag, which every dependency wait of the launch checks, and waits for
// the launch to drain.
void wait_run(qs_batch *b)
{
    hipchk(hipEventRecord(b->done_ev, b->stream), "hipEventRecord");
    const auto t0 = std::chrono::steady_clock::now();
    const double limit_s = 60.0 + 4.0 * (b->opts.wait_ms > 0 ? b->opts.wait_ms : 2000) / 1000.0;
    for (;;) {
        const hipError_t e = hipEventQuery(b->done_ev);
        if (e == hipSuccess)
            break;
        if (e != hipErrorNotReady)
            hipchk(e, "hipEventQuery");
        if (std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() > limit_s) {
            __atomic_store_n(&b->h_flags[0], 1u, __ATOMIC_SEQ_CST);
            hipchk(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
            __atomic_store_n(&b->h_flags[0], 0u, __ATOMIC_SEQ_CST);
            fail(QS_ERR_HIP, "batch run did not finish in time; its waits were aborted");
        }
        std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
    if (__atomic_load_n(&b->h_flags[1], __ATOMIC_SEQ_CST) != 0u) {
        __atomic_store_n(&b->h_flags[1], 0u, __ATOMIC_SEQ_CST);
        fail(QS_ERR_HIP, "a work item of the batch launch waited too long for its circuit's previous pass");
    }
}

}  // namespace

extern "C" {

qs_status qs_batch_plan(int count, const int *n_qubits, const qs_gate *const *gates, const int64_t *n_gates,
                        qs_dtype dt, const qs_batch_opts *opts, qs_batch_pass_info *passes, int64_t pass_cap,
                        int64_t *n_passes, qs_batch_item_info *items, int64_t item_cap, int64_t *n_items)
{
    return guard([&] {
        if (count < 1 || !n_qubits || !gates || !n_gates || !opts || !n_passes || !n_items)
            fail(QS_ERR_ARG, "bad arguments");
        if (dt != QS_C64 && dt != QS_C128)
            fail(QS_ERR_ARG, "unknown dtype");
        BatchPlan bp;
        plan_batch(count, n_qubits, gates, n_gates, dt, *opts, bp);
        *n_passes = (int64_t)bp.passes.size();
        *n_items = (int64_t)bp.items.size();
        for (int64_t i = 0; passes && i < pass_cap && i < *n_passes; ++i) {
            const PlanPass &P = bp.passes[i];
            passes[i] = qs_batch_pass_info{P.circuit, P.level, P.k, P.last, (int64_t)P.tiles};
        }
        for (int64_t i = 0; items && i < item_cap && i < *n_items; ++i) {
            const QueueItem &it = bp.items[i];
            items[i] = qs_batch_item_info{(int32_t)it.pass, it.dep, (int64_t)it.t0, (int64_t)it.t1,
                                          (int64_t)it.need};
        }
    });
}

qs_status qs_batch_create(int count, const int *n_qubits, const qs_gate *const *gates, const int64_t *n_gates,
                          qs_dtype dt, const qs_batch_opts *opts, qs_batch **out)
{
    return guard([&] {
        if (!out || count < 1 || !n_qubits || !gates || !n_gates || !opts)
            fail(QS_ERR_ARG, "bad arguments");
        *out = nullptr;
        if (dt != QS_C64 && dt != QS_C128)
            fail(QS_ERR_ARG, "unknown dtype");
        const qs_batch_opts o = *opts;
        const size_t eb = dt == QS_C64 ? 8 : 16;
        auto t0 = std::chrono::steady_clock::now();
        BatchPlan bp;
        plan_batch(count, n_qubits, gates, n_gates, dt, o, bp);
        auto *b = new qs_batch();
        try {
            b->count = count;
            b->dt = dt;
            b->opts = o;
            b->n.assign(n_qubits, n_qubits + count);
            b->start.resize(count);
            for (int c = 0; c < count; ++c) {
                b->start[c] = b->total;
                b->total += 1ull << b->n[c];
            }
            hipchk(hipMalloc(&b->d_state, b->total * eb), "hipMalloc(batch states)");
            std::vector<size_t> op_base(count, 0);
            std::vector<TileOp> ops;
            for (int c = 0; c < count; ++c) {
                op_base[c] = ops.size();
                ops.insert(ops.end(), bp.progs[c].ops.begin(), bp.progs[c].ops.end());
            }
            upload(b->d_ops, ops, "batch ops");
            // read-out partials: two per tile of each circuit's last pass
            for (int c = 0; c < count; ++c) {
                b->part_off.push_back(b->n_partials);
                b->part_cnt.push_back((uint32_t)(1ull << (b->n[c] - bp.k[c])));
                b->n_partials += b->part_cnt.back();
            }
            for (const PlanPass &P : bp.passes) {
                const int c = P.circuit;
                BatchPass D{};
                if (P.launch) {
                    tile_args_from_launch(*P.launch, D.t);
                    D.t.ops = b->d_ops + op_base[c] + P.launch->op_begin;
                } else {
                    tile_args_identity(P.k, QUEUE_LOG_NT, P.k - QUEUE_LOG_NT, D.t);
                    D.t.ops = b->d_ops;
                }
                D.t.state = static_cast<char *>(b->d_state) + b->start[c] * eb;
                D.t.n_hi = b->n[c] - P.k;
                if (P.level == 0)
                    D.t.io |= IO_BASIS;  // the first pass starts from |0...0> instead of reading the state
                D.ntiles = P.tiles;
                D.last = P.last;
                D.zpos = bp.progs[c].sigma_final[0];
                D.circuit = c;
                D.part = b->part_off[c];
                b->passes.push_back(D);
                b->stats.n_tiles += P.tiles;
            }
            b->items = bp.items;
            for (int c = 0; c < count; ++c) {
                b->stats.n_gates += bp.progs[c].stats.n_gates;
                b->stats.n_perm += bp.progs[c].stats.n_perm;
            }
            b->stats.n_passes = (int64_t)bp.passes.size();
            b->stats.n_items = (int64_t)b->items.size();
            upload(b->d_passes, b->passes, "batch passes");
            upload(b->d_items, b->items, "batch items");
            upload(b->d_part_off, b->part_off, "batch partial offsets");
            upload(b->d_part_cnt, b->part_cnt, "batch partial counts");
            b->n_words = 4 + b->passes.size();
            hipchk(hipMalloc(&b->d_words, b->n_words * sizeof(uint32_t)), "hipMalloc(batch counters)");
            hipchk(hipMalloc(&b->d_partials, std::max<uint64_t>(1, b->n_partials) * 2 * sizeof(double)),
                   "hipMalloc(partials)");
            hipchk(hipMalloc(&b->d_out, (size_t)count * 2 * sizeof(double)), "hipMalloc(batch out)");
            hipchk(hipHostMalloc(reinterpret_cast<void **>(&b->h_flags), 4 * sizeof(uint32_t), hipHostMallocCoherent),
                   "hipHostMalloc(batch flags)");
            std::memset(b->h_flags, 0, 4 * sizeof(uint32_t));
            hipchk(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking), "hipStreamCreate");
            hipchk(hipEventCreateWithFlags(&b->done_ev, hipEventDisableTiming), "hipEventCreate");
            int dev = 0, cus = 0;
            hipchk(hipGetDevice(&dev), "hipGetDevice");
            hipchk(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "hipDeviceGetAttribute");
            b->grid = std::max(1, cus * (o.wg_per_cu > 0 ? o.wg_per_cu : 4));
            b->stats.state_bytes = (double)(b->total * eb);
        } catch (...) {
            free_batch(b);
            delete b;
            throw;
        }
        auto t1 = std::chrono::steady_clock::now();
        b->stats.compile_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
        *out = b;
    });
}

qs_status qs_batch_run(qs_batch *b)
{
    return guard([&] {
        if (!b)
            fail(QS_ERR_ARG, "batch is NULL");
        if (!b->opts.use_graph) {
            enqueue(b);
            return;
        }
        if (!b->exec) {
            hipchk(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
            try {
                enqueue(b);
            } catch (...) {
                hipGraph_t g = nullptr;
                (void)hipStreamEndCapture(b->stream, &g);
                if (g)
                    (void)hipGraphDestroy(g);
                throw;
            }
            hipchk(hipStreamEndCapture(b->stream, &b->graph), "hipStreamEndCapture");
            hipchk(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
        }
        hipchk(hipGraphLaunch(b->exec, b->stream), "hipGraphLaunch");
    });
}

qs_status qs_batch_results(qs_batch *b, double *z0, double *norms)
{
    return guard([&] {
        if (!b)
            fail(QS_ERR_ARG, "batch is NULL");
        wait_run(b);
        std::vector<double> out((size_t)b->count * 2);
        hipchk(hipMemcpyAsync(out.data(), b->d_out, out.size() * sizeof(double), hipMemcpyDeviceToHost, b->stream),
               "hipMemcpyAsync");
        hipchk(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
        for (int c = 0; c < b->count; ++c) {
            if (z0)
                z0[c] = out[2 * c];
            if (norms)
                norms[c] = out[2 * c + 1];
        }
    });
}

qs_status qs_batch_read_state(qs_batch *b, int circuit, double *out)
{
    return guard([&] {
        if (!b || !out || circuit < 0 || circuit >= b->count)
            fail(QS_ERR_ARG, "bad arguments");
        const int n = b->n[circuit];
        if (n > 26)
            fail(QS_ERR_ARG, "qs_batch_read_state is limited to n <= 26");
        wait_run(b);
        // placements are relabelled, so every state stays in its starting
        // (identity) placement: physical order is logical order
        const uint64_t N = 1ull << n;
        const size_t eb = b->dt == QS_C64 ? 8 : 16;
        std::vector<unsigned char> raw(N * eb);
        hipchk(hipMemcpyAsync(raw.data(), static_cast<char *>(b->d_state) + b->start[circuit] * eb, raw.size(),
                              hipMemcpyDeviceToHost, b->stream),
               "hipMemcpyAsync");
        hipchk(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
        for (uint64_t i = 0; i < N; ++i) {
            if (b->dt == QS_C64) {
                const float *f = reinterpret_cast<const float *>(raw.data());
                out[2 * i] = f[2 * i];
                out[2 * i + 1] = f[2 * i + 1];
            } else {
                const double *d = reinterpret_cast<const double *>(raw.data());
                out[2 * i] = d[2 * i];
                out[2 * i + 1] = d[2 * i + 1];
            }
        }
    });
}

qs_status qs_batch_get_stats(const qs_batch *b, qs_batch_stats *out)
{
    return guard([&] {
        if (!b || !out)
            fail(QS_ERR_ARG, "bad arguments");
        *out = b->stats;
    });
}

qs_status qs_batch_synchronize(qs_batch *b)
{
    return guard([&] {
        if (!b)
            fail(QS_ERR_ARG, "batch is NULL");
        wait_run(b);
    });
}

qs_status qs_batch_destroy(qs_batch *b)
{
    return guard([&] {
        if (!b)
            return;
        if (b->stream)
            (void)hipStreamSynchronize(b->stream);  // a run in flight drains (its waits are bounded)
        free_batch(b);
        delete b;
    });
}

}  // extern "C"
