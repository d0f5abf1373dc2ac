// Batching form (C boundary): many independent circuits of different sizes
// compiled together and executed level by level (one persistent launch per
// pass level), the whole sequence captured once in a HIP graph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"
#include "kernels.h"

using namespace qsim;

struct qs_batch {
    int count = 0;
    qs_dtype dt = QS_C64;
    qs_batch_opts opts{};
    int log_r = 0, log_nt = 0, grid = 0;
    hipStream_t stream = nullptr;
    std::vector<int> n;
    std::vector<uint64_t> start;  // element offset of each state
    uint64_t total = 0;
    std::vector<BatchPass> passes;
    std::vector<BatchItem> items;
    std::vector<uint32_t> level_start;  // items of level L: [level_start[L], level_start[L+1])
    std::vector<std::vector<int>> circ_passes;  // pass indices of each circuit, in order
    std::vector<std::vector<int>> level_solo;   // passes of level L run as launches of their own
    uint64_t solo_tiles = 1ull << 12;           // 0: every pass in the level launch
    size_t items_cap = 0;                       // BatchItem capacity of d_items
    std::vector<TileOp> ops;
    std::vector<uint64_t> part_off;
    std::vector<uint32_t> part_cnt;
    uint64_t n_partials = 0;
    // device
    void *d_state = nullptr;
    TileOp *d_ops = nullptr;
    BatchPass *d_passes = nullptr;
    BatchItem *d_items = nullptr;
    double *d_partials = nullptr, *d_out = nullptr;
    uint64_t *d_starts = nullptr, *d_part_off = nullptr;
    uint32_t *d_part_cnt = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    qs_batch_stats stats{};
};

namespace {

void hipchk(hipError_t e, const char *what)
{
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(e == hipErrorOutOfMemory ? QS_ERR_OOM : QS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
    }
}

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
    void *ptrs[] = {b->d_state, b->d_ops, b->d_passes, b->d_items, b->d_partials,
                    b->d_out, b->d_starts, b->d_part_off, b->d_part_cnt};
    for (void *p : ptrs)
        if (p)
            (void)hipFree(p);
    if (b->stream)
        (void)hipStreamDestroy(b->stream);
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

// Work items of each pass level.  A pass of at least solo_tiles tiles that is
// not its circuit's last (the last one also produces the read-out partials)
// goes to level_solo instead: it fills the device by itself and runs as a
// tile-pass launch (one workgroup per tile) after the level launch.
void build_levels(qs_batch *b)
{
    const uint32_t chunk = (uint32_t)std::max(1, b->opts.chunk);
    size_t max_np = 0;
    for (auto &v : b->circ_passes)
        max_np = std::max(max_np, v.size());
    b->items.clear();
    b->level_start.clear();
    b->level_solo.assign(max_np, {});
    for (size_t lvl = 0; lvl < max_np; ++lvl) {
        b->level_start.push_back((uint32_t)b->items.size());
        for (int c = 0; c < b->count; ++c) {
            if (lvl >= b->circ_passes[c].size())
                continue;
            const int pi = b->circ_passes[c][lvl];
            const BatchPass &P = b->passes[pi];
            const uint32_t nt = P.ntiles;
            if (b->solo_tiles && nt >= b->solo_tiles && !P.last) {
                b->level_solo[lvl].push_back(pi);
                continue;
            }
            for (uint32_t t = 0; t < nt; t += chunk)
                b->items.push_back(BatchItem{(uint32_t)pi, t, std::min(nt, t + chunk), 0});
        }
    }
    b->level_start.push_back((uint32_t)b->items.size());
    b->stats.n_items = (int64_t)b->items.size();
}

void enqueue(qs_batch *b)
{
    launch_batch_init(b->d_state, b->dt, b->total, b->d_starts, b->count, b->stream);
    for (size_t L = 0; L + 1 < b->level_start.size(); ++L) {
        BatchArgs a{};
        a.passes = b->d_passes;
        a.items = b->d_items;
        a.i0 = b->level_start[L];
        a.i1 = b->level_start[L + 1];
        a.partials = b->d_partials;
        const int grid = (int)std::min<uint32_t>((uint32_t)b->grid, a.i1 - a.i0);
        if (grid > 0) {
            if (b->dt == QS_C64)
                launch_batch_f32(a, b->log_r, b->log_nt, grid, b->stream);
            else
                launch_batch_f64(a, b->log_r, b->log_nt, grid, b->stream);
        }
        for (int pi : b->level_solo[L]) {
            const BatchPass &P = b->passes[pi];
            if (b->dt == QS_C64)
                launch_tile_f32(P.t, P.ntiles, b->log_r, b->log_nt, b->stream);
            else
                launch_tile_f64(P.t, P.ntiles, b->log_r, b->log_nt, b->stream);
        }
    }
    launch_batch_reduce(b->d_partials, b->d_part_off, b->d_part_cnt, b->count, b->d_out, b->stream);
}

}  // namespace

extern "C" {

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
        const int K = o.k_tile;
        const size_t eb = dt == QS_C64 ? 8 : 16;
        if (K < MIN_TILE_BITS || (eb << K) > MAX_BATCH_TILE_BYTES)
            fail(QS_ERR_ARG, "k_tile out of range for the batching form");
        for (int c = 0; c < count; ++c)
            if (n_qubits[c] < K || n_qubits[c] > MAX_QUBITS)
                fail(QS_ERR_ARG, "every circuit needs k_tile <= n <= 34 (circuit " + std::to_string(c) + ")");
        auto t0 = std::chrono::steady_clock::now();
        auto *b = new qs_batch();
        try {
            b->count = count;
            b->dt = dt;
            b->opts = o;
            tile_shape(K, dt, o.reg_bits, &b->log_r, &b->log_nt);
            b->n.assign(n_qubits, n_qubits + count);
            b->start.resize(count);
            for (int c = 0; c < count; ++c) {
                b->start[c] = b->total;
                b->total += 1ull << b->n[c];
            }
            // compile every circuit (host threads)
            std::vector<Program> progs(count);
            qs_run_opts ro{};
            ro.form = QS_FORM_PASS;
            ro.k_tile = K;
            ro.max_swaps = std::max(1, o.max_swaps);
            ro.pinned = std::min(o.pinned, K);
            ro.perm_exec = QS_PERM_RELABEL;
            ro.max_fuse = o.max_fuse;
            ro.reg_bits = b->log_r;
            std::vector<std::string> errs(count);
            const unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
            std::vector<std::thread> th;
            for (unsigned w = 0; w < nth; ++w)
                th.emplace_back([&, w] {
                    for (int c = (int)w; c < count; c += (int)nth) {
                        try {
                            compile_program(gates[c], n_gates[c], b->n[c], dt, nullptr, ro, progs[c]);
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

            // device buffers whose addresses the pass table needs
            hipchk(hipMalloc(&b->d_state, b->total * eb), "hipMalloc(batch states)");
            size_t n_ops = 0;
            for (auto &p : progs)
                n_ops += p.ops.size();
            hipchk(hipMalloc(&b->d_ops, std::max<size_t>(1, n_ops) * sizeof(TileOp)), "hipMalloc(batch ops)");

            // pass table: each circuit's tile passes; a circuit without gates
            // gets one empty pass so that its read-out is still produced
            std::vector<std::vector<int>> circ_passes(count);
            size_t op_base = 0;
            for (int c = 0; c < count; ++c) {
                Program &p = progs[c];
                const uint64_t ntiles = 1ull << (b->n[c] - K);
                std::vector<const Launch *> tl;
                for (const Launch &L : p.launches) {
                    if (L.type != L_TILE)
                        fail(QS_ERR_UNSUPPORTED, "batch circuit " + std::to_string(c) + " needs a non-tile launch");
                    tl.push_back(&L);
                }
                const int np = std::max<int>(1, (int)tl.size());
                b->part_off.push_back(b->n_partials);
                b->part_cnt.push_back((uint32_t)ntiles);
                for (int i = 0; i < np; ++i) {
                    BatchPass P{};
                    P.t.state = static_cast<char *>(b->d_state) + b->start[c] * eb;
                    if (!tl.empty()) {
                        tile_args_from_launch(*tl[i], P.t);
                        P.t.ops = b->d_ops + op_base + tl[i]->op_begin;
                    } else {
                        tile_args_identity(K, b->log_nt, b->log_r, P.t);
                        P.t.ops = b->d_ops;
                    }
                    P.t.n_hi = b->n[c] - K;
                    P.ntiles = (uint32_t)ntiles;
                    P.last = i == np - 1;
                    P.zpos = p.sigma_final[0];
                    P.part = b->n_partials;
                    circ_passes[c].push_back((int)b->passes.size());
                    b->passes.push_back(P);
                }
                b->n_partials += ntiles;
                b->ops.insert(b->ops.end(), p.ops.begin(), p.ops.end());
                op_base += p.ops.size();
                b->stats.n_passes += np;
                b->stats.n_tiles += (int64_t)np * (int64_t)ntiles;
                b->stats.n_gates += p.stats.n_gates;
                b->stats.n_perm += p.stats.n_perm;
            }
            // work items ordered by pass level
            b->circ_passes = std::move(circ_passes);
            build_levels(b);
            b->items_cap = std::max<size_t>(1, b->items.size());

            if (!b->ops.empty())
                hipchk(hipMemcpy(b->d_ops, b->ops.data(), b->ops.size() * sizeof(TileOp), hipMemcpyHostToDevice),
                       "hipMemcpy(batch ops)");
            upload(b->d_passes, b->passes, "batch passes");
            upload(b->d_items, b->items, "batch items");
            upload(b->d_starts, b->start, "batch starts");
            upload(b->d_part_off, b->part_off, "batch partial offsets");
            upload(b->d_part_cnt, b->part_cnt, "batch partial counts");
            hipchk(hipMalloc(&b->d_partials, std::max<uint64_t>(1, b->n_partials) * 2 * sizeof(double)),
                   "hipMalloc(partials)");
            hipchk(hipMalloc(&b->d_out, (size_t)count * 2 * sizeof(double)), "hipMalloc(batch out)");
            hipchk(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking), "hipStreamCreate");
            int dev = 0, cus = 0;
            hipchk(hipGetDevice(&dev), "hipGetDevice");
            hipchk(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "hipDeviceGetAttribute");
            b->grid = std::max(1, cus * std::max(1, o.wg_per_cu));
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

qs_status qs_batch_set_solo_tiles(qs_batch *b, int64_t min_tiles)
{
    return guard([&] {
        if (!b || min_tiles < 0)
            fail(QS_ERR_ARG, "bad arguments");
        hipchk(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
        b->solo_tiles = (uint64_t)min_tiles;
        build_levels(b);
        if (b->items.size() > b->items_cap) {
            hipchk(hipFree(b->d_items), "hipFree(batch items)");
            b->d_items = nullptr;
            hipchk(hipMalloc(&b->d_items, b->items.size() * sizeof(BatchItem)), "hipMalloc(batch items)");
            b->items_cap = b->items.size();
        }
        if (!b->items.empty())
            hipchk(hipMemcpy(b->d_items, b->items.data(), b->items.size() * sizeof(BatchItem),
                             hipMemcpyHostToDevice),
                   "hipMemcpy(batch items)");
        // the captured launch sequence no longer matches: capture again at the next run
        if (b->exec)
            hipchk(hipGraphExecDestroy(b->exec), "hipGraphExecDestroy");
        b->exec = nullptr;
        if (b->graph)
            hipchk(hipGraphDestroy(b->graph), "hipGraphDestroy");
        b->graph = nullptr;
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
        hipchk(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    });
}

qs_status qs_batch_destroy(qs_batch *b)
{
    return guard([&] {
        if (!b)
            return;
        (void)hipStreamSynchronize(b->stream);
        free_batch(b);
        delete b;
    });
}

}  // extern "C"
