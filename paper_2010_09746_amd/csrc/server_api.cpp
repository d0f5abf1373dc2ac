// Serving form (C boundary): resident request states advanced by continuous
// batching.  Each step is one launch of the level kernel of the batching form
// over the next tile pass of every resident request; a request's read-out
// (<Z_q> for all q, sampled amplitudes, norm) is enqueued right after its last
// pass and copied to pinned host memory within the same step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "internal.h"
#include "kernels.h"

using namespace qsim;

namespace {

// First-fit allocator of unit ranges [0, cap), coalescing on release.
class RangeAlloc {
public:
    void init(uint64_t cap)
    {
        free_.clear();
        if (cap)
            free_[0] = cap;
    }
    bool alloc(uint64_t n, uint64_t align, uint64_t *off)
    {
        n = std::max<uint64_t>(n, 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            const uint64_t s = it->first, len = it->second;
            const uint64_t a = (s + align - 1) / align * align;
            if (a + n > s + len)
                continue;
            free_.erase(it);
            if (a > s)
                free_[s] = a - s;
            if (a + n < s + len)
                free_[a + n] = s + len - (a + n);
            *off = a;
            return true;
        }
        return false;
    }
    void release(uint64_t off, uint64_t n)
    {
        n = std::max<uint64_t>(n, 1);
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

private:
    std::map<uint64_t, uint64_t> free_;
};

struct SReq {
    int64_t id = 0;
    int n = 0;
    void *state = nullptr;
    size_t bytes = 0;
    std::vector<TileOp> ops;
    std::vector<BatchPass> passes;
    std::vector<uint64_t> samples;
    uint64_t ops_off = 0, ops_len = 0, samp_off = 0, samp_len = 0, res_off = 0, res_len = 0;
    uint64_t pass_off = 0, np = 0;
    uint64_t cur = 0;
    int slot = -1;  // pinned result slot
    bool done = false;
    std::vector<double> res;  // norm, S_0..S_{n-1}, amplitudes
};

constexpr uint64_t ARENA_BYTES = 256ull << 20;
constexpr uint64_t PASS_RECORDS = 1ull << 20;

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

// One enqueued step: the requests whose last pass (and read-out) it runs and
// the event recorded after its work.
struct SStep {
    std::vector<int64_t> finishing;
    hipEvent_t ev = nullptr;
    BatchItem *d_items = nullptr, *h_items = nullptr;  // this step's work items (device, pinned staging)
    size_t items_cap = 0;
};

constexpr int MAX_STEPS_IN_FLIGHT = 2;
constexpr int SIDE_STREAMS = 3;  // with the server's own stream: 4, the device's hardware queues

struct qs_server {
    qs_dtype dt = QS_C64;
    qs_batch_opts opts{};
    int K = 0, log_r = 0, log_nt = 0, grid = 0;
    size_t budget = 0, resident = 0;
    int max_slots = 0, max_samples = 0;
    hipStream_t stream = nullptr;
    // large requests' passes of a step run on these, forked from and joined
    // back into the server's stream
    hipStream_t side[SIDE_STREAMS] = {};
    hipEvent_t fork_ev = nullptr, join_ev[SIDE_STREAMS] = {};
    SStep steps[MAX_STEPS_IN_FLIGHT];
    int step_head = 0, steps_pending = 0;  // oldest pending step, number pending
    char *d_bytes = nullptr;
    RangeAlloc bytes_alloc;
    BatchPass *d_passes = nullptr;
    RangeAlloc pass_alloc;
    double *d_zwork = nullptr;
    double *h_res = nullptr;  // pinned: max_slots slots of res_stride doubles
    size_t res_stride = 0;
    std::vector<int> free_slots;
    std::map<int64_t, SReq> reqs;
    std::vector<int64_t> active;  // admission order
    int64_t next_id = 1;
    // a request whose pass has at least this many tiles runs it as a tile-pass
    // launch of its own (one workgroup per tile) inside the step; 0: never
    uint64_t solo_tiles = 1ull << 10;
};

namespace {

void destroy_server(qs_server *s)
{
    if (s->stream)
        (void)hipStreamSynchronize(s->stream);
    for (auto &st : s->steps)
        if (st.ev)
            (void)hipEventDestroy(st.ev);
    if (s->fork_ev)
        (void)hipEventDestroy(s->fork_ev);
    for (int i = 0; i < SIDE_STREAMS; ++i) {
        if (s->join_ev[i])
            (void)hipEventDestroy(s->join_ev[i]);
        if (s->side[i]) {
            (void)hipStreamSynchronize(s->side[i]);
            (void)hipStreamDestroy(s->side[i]);
        }
    }
    void *dev[] = {s->d_bytes, s->d_passes, s->d_zwork};
    for (void *p : dev)
        if (p)
            (void)hipFree(p);
    for (auto &st : s->steps) {
        if (st.d_items)
            (void)hipFree(st.d_items);
        if (st.h_items)
            (void)hipHostFree(st.h_items);
    }
    if (s->h_res)
        (void)hipHostFree(s->h_res);
    if (s->stream)
        (void)hipStreamDestroy(s->stream);
}

// Grow a step's item buffers; the step's previous use has been waited for.
void ensure_items(SStep &st, size_t need)
{
    if (need <= st.items_cap)
        return;
    size_t cap = std::max<size_t>(need, 2 * st.items_cap);
    if (st.d_items)
        hipchk(hipFree(st.d_items), "hipFree");
    if (st.h_items)
        hipchk(hipHostFree(st.h_items), "hipHostFree");
    st.d_items = nullptr;
    st.h_items = nullptr;
    st.items_cap = 0;
    hipchk(hipMalloc(&st.d_items, cap * sizeof(BatchItem)), "hipMalloc(items)");
    hipchk(hipHostMalloc(reinterpret_cast<void **>(&st.h_items), cap * sizeof(BatchItem), hipHostMallocDefault),
           "hipHostMalloc(items)");
    st.items_cap = cap;
}

}  // namespace

extern "C" {

qs_status qs_server_create(qs_dtype dt, const qs_batch_opts *opts, size_t hbm_budget, int max_slots,
                           int max_samples, qs_server **out)
{
    return guard([&] {
        if (!out || !opts || max_slots < 1 || max_slots > 4096 || max_samples < 0 || max_samples > 4096)
            fail(QS_ERR_ARG, "bad arguments");
        if (dt != QS_C64 && dt != QS_C128)
            fail(QS_ERR_ARG, "unknown dtype");
        *out = nullptr;
        const size_t eb = dt == QS_C64 ? 8 : 16;
        if (opts->k_tile < MIN_TILE_BITS || (eb << opts->k_tile) > MAX_BATCH_TILE_BYTES)
            fail(QS_ERR_ARG, "k_tile out of range");
        auto *s = new qs_server();
        try {
            s->dt = dt;
            s->opts = *opts;
            s->K = opts->k_tile;
            tile_shape(s->K, dt, opts->reg_bits, &s->log_r, &s->log_nt);
            s->budget = hbm_budget;
            s->max_slots = max_slots;
            s->max_samples = max_samples;
            hipchk(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking), "hipStreamCreate");
            for (auto &st : s->steps)
                hipchk(hipEventCreateWithFlags(&st.ev, hipEventDisableTiming), "hipEventCreate");
            hipchk(hipEventCreateWithFlags(&s->fork_ev, hipEventDisableTiming), "hipEventCreate");
            for (int i = 0; i < SIDE_STREAMS; ++i) {
                hipchk(hipStreamCreateWithFlags(&s->side[i], hipStreamNonBlocking), "hipStreamCreate");
                hipchk(hipEventCreateWithFlags(&s->join_ev[i], hipEventDisableTiming), "hipEventCreate");
            }
            hipchk(hipMalloc(&s->d_bytes, ARENA_BYTES), "hipMalloc(server arena)");
            s->bytes_alloc.init(ARENA_BYTES);
            hipchk(hipMalloc(&s->d_passes, PASS_RECORDS * sizeof(BatchPass)), "hipMalloc(server passes)");
            s->pass_alloc.init(PASS_RECORDS);
            hipchk(hipMalloc(&s->d_zwork, zsum_work_doubles(MAX_QUBITS) * sizeof(double)), "hipMalloc(read-out)");
            s->res_stride = (size_t)(MAX_QUBITS + 1) + 2 * (size_t)max_samples;
            hipchk(hipHostMalloc(reinterpret_cast<void **>(&s->h_res), s->res_stride * max_slots * sizeof(double),
                                 hipHostMallocDefault),
                   "hipHostMalloc(results)");
            for (int i = max_slots - 1; i >= 0; --i)
                s->free_slots.push_back(i);
            int dev = 0, cus = 0;
            hipchk(hipGetDevice(&dev), "hipGetDevice");
            hipchk(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "hipDeviceGetAttribute");
            s->grid = std::max(1, cus * std::max(1, opts->wg_per_cu));
            for (auto &st : s->steps)
                ensure_items(st, 4096);
        } catch (...) {
            destroy_server(s);
            delete s;
            throw;
        }
        *out = s;
    });
}

qs_status qs_server_set_solo_tiles(qs_server *s, int64_t min_tiles)
{
    return guard([&] {
        if (!s || min_tiles < 0)
            fail(QS_ERR_ARG, "bad arguments");
        if (s->steps_pending)
            fail(QS_ERR_STATE, "a step is in flight");
        s->solo_tiles = (uint64_t)min_tiles;
    });
}

qs_status qs_server_destroy(qs_server *s)
{
    return guard([&] {
        if (!s)
            return;
        destroy_server(s);
        delete s;
    });
}

qs_status qs_server_fits(const qs_server *s, int n, int *fits)
{
    return guard([&] {
        if (!s || !fits)
            fail(QS_ERR_ARG, "bad arguments");
        const size_t bytes = (size_t)(s->dt == QS_C64 ? 8 : 16) << n;
        *fits = (s->resident + bytes <= s->budget) && !s->free_slots.empty() ? 1 : 0;
    });
}

qs_status qs_server_admit(qs_server *s, const qs_program *pp, void *state_buf, size_t buf_bytes,
                          const uint64_t *samples, int count, int64_t *request_id)
{
    return guard([&] {
        if (!s || !pp || !state_buf || !request_id || count < 0 || count > s->max_samples || (count && !samples))
            fail(QS_ERR_ARG, "bad arguments");
        const Program &p = pp->p;
        const int n = p.n;
        const size_t eb = s->dt == QS_C64 ? 8 : 16;
        const size_t bytes = eb << n;
        if (p.dt != s->dt)
            fail(QS_ERR_ARG, "program compiled for another amplitude type");
        if (n < s->K || n > MAX_QUBITS)
            fail(QS_ERR_ARG, "request needs k_tile <= n <= 34");
        if (buf_bytes < bytes)
            fail(QS_ERR_ARG, "state buffer smaller than 2^n amplitudes");
        for (int q = 0; q < n; ++q)
            if (p.sigma0[q] != q)
                fail(QS_ERR_ARG, "program must start from the identity placement");
        for (int i = 0; i < count; ++i)
            if (samples[i] >= (1ull << n))
                fail(QS_ERR_ARG, "sample index out of range");
        if (s->resident + bytes > s->budget || s->free_slots.empty())
            fail(QS_ERR_BUDGET, "request does not fit the memory budget or the slots");
        SReq r;
        r.id = s->next_id;
        r.n = n;
        r.state = state_buf;
        r.bytes = bytes;
        r.ops = p.ops;
        std::vector<const Launch *> tl;
        for (const Launch &L : p.launches) {
            if (L.type != L_TILE || L.k != s->K || L.log_r != s->log_r)
                fail(QS_ERR_ARG, "program not compiled with this server's tile options (relabel, k_tile, reg_bits)");
            tl.push_back(&L);
        }
        r.np = std::max<size_t>(1, tl.size());
        // arena space: ops, samples, read-out
        r.ops_len = std::max<size_t>(1, r.ops.size()) * sizeof(TileOp);
        r.samp_len = std::max(1, count) * sizeof(uint64_t);
        r.res_len = ((size_t)n + 1 + 2 * (size_t)count) * sizeof(double);
        const bool a1 = s->bytes_alloc.alloc(r.ops_len, 256, &r.ops_off);
        const bool a2 = a1 && s->bytes_alloc.alloc(r.samp_len, 256, &r.samp_off);
        const bool a3 = a2 && s->bytes_alloc.alloc(r.res_len, 256, &r.res_off);
        const bool a4 = a3 && s->pass_alloc.alloc(r.np, 1, &r.pass_off);
        if (!a4) {
            if (a1)
                s->bytes_alloc.release(r.ops_off, r.ops_len);
            if (a2)
                s->bytes_alloc.release(r.samp_off, r.samp_len);
            if (a3)
                s->bytes_alloc.release(r.res_off, r.res_len);
            fail(QS_ERR_BUDGET, "server arena exhausted");
        }
        TileOp *d_ops = reinterpret_cast<TileOp *>(s->d_bytes + r.ops_off);
        const uint64_t ntiles = 1ull << (n - s->K);
        for (uint64_t i = 0; i < r.np; ++i) {
            BatchPass P{};
            P.t.state = state_buf;
            if (!tl.empty()) {
                tile_args_from_launch(*tl[i], P.t);
                P.t.ops = d_ops + tl[i]->op_begin;
            } else {
                tile_args_identity(s->K, s->log_nt, s->log_r, P.t);
                P.t.ops = d_ops;
            }
            P.t.n_hi = n - s->K;
            P.ntiles = (uint32_t)ntiles;
            P.last = 0;
            P.zpos = 0;
            r.passes.push_back(P);
        }
        r.samples.assign(samples, samples + count);
        if (!r.ops.empty())
            hipchk(hipMemcpyAsync(d_ops, r.ops.data(), r.ops.size() * sizeof(TileOp), hipMemcpyHostToDevice,
                                  s->stream),
                   "hipMemcpyAsync(ops)");
        hipchk(hipMemcpyAsync(s->d_passes + r.pass_off, r.passes.data(), r.passes.size() * sizeof(BatchPass),
                              hipMemcpyHostToDevice, s->stream),
               "hipMemcpyAsync(passes)");
        if (count)
            hipchk(hipMemcpyAsync(s->d_bytes + r.samp_off, r.samples.data(), count * sizeof(uint64_t),
                                  hipMemcpyHostToDevice, s->stream),
                   "hipMemcpyAsync(samples)");
        launch_set_basis(state_buf, s->dt, n, 0, s->stream);
        r.slot = s->free_slots.back();
        s->free_slots.pop_back();
        s->resident += bytes;
        *request_id = r.id;
        s->active.push_back(r.id);
        s->reqs.emplace(r.id, std::move(r));
        ++s->next_id;
    });
}

qs_status qs_server_step_launch(qs_server *s, int *n_running)
{
    return guard([&] {
        if (!s)
            fail(QS_ERR_ARG, "server is NULL");
        if (s->steps_pending >= MAX_STEPS_IN_FLIGHT)
            fail(QS_ERR_STATE, "two steps in flight: wait for the older one first");
        SStep &step = s->steps[(s->step_head + s->steps_pending) % MAX_STEPS_IN_FLIGHT];
        const uint32_t chunk = (uint32_t)std::max(1, s->opts.chunk);
        size_t need = 0;
        for (int64_t id : s->active) {
            const SReq &r = s->reqs.at(id);
            if (r.cur < r.np)
                need += ((1ull << (r.n - s->K)) + chunk - 1) / chunk;
        }
        ensure_items(step, need + 1);
        size_t ni = 0;
        int running = 0;
        step.finishing.clear();
        std::vector<const BatchPass *> solo;
        for (int64_t id : s->active) {
            SReq &r = s->reqs.at(id);
            if (r.cur >= r.np)
                continue;
            const uint32_t pi = (uint32_t)(r.pass_off + r.cur);
            const uint32_t nt = (uint32_t)(1ull << (r.n - s->K));
            if (s->solo_tiles && nt >= s->solo_tiles) {
                solo.push_back(&r.passes[r.cur]);
            } else {
                for (uint32_t t = 0; t < nt; t += chunk)
                    step.h_items[ni++] = BatchItem{pi, t, std::min(nt, t + chunk), 0};
            }
            ++r.cur;
            ++running;
            if (r.cur == r.np)
                step.finishing.push_back(id);
        }
        // the large passes start with the shared launch: each request appears
        // once in a step, so they are independent of it
        const int ns = std::min<int>(SIDE_STREAMS, (int)solo.size());
        if (ns) {
            hipchk(hipEventRecord(s->fork_ev, s->stream), "hipEventRecord");
            for (int i = 0; i < ns; ++i)
                hipchk(hipStreamWaitEvent(s->side[i], s->fork_ev, 0), "hipStreamWaitEvent");
        }
        if (ni) {
            hipchk(hipMemcpyAsync(step.d_items, step.h_items, ni * sizeof(BatchItem), hipMemcpyHostToDevice,
                                  s->stream),
                   "hipMemcpyAsync(items)");
            BatchArgs a{};
            a.passes = s->d_passes;
            a.items = step.d_items;
            a.i0 = 0;
            a.i1 = (uint32_t)ni;
            a.partials = nullptr;
            const int grid = (int)std::min<size_t>((size_t)s->grid, ni);
            if (s->dt == QS_C64)
                launch_batch_f32(a, s->log_r, s->log_nt, grid, s->stream);
            else
                launch_batch_f64(a, s->log_r, s->log_nt, grid, s->stream);
        }
        // large passes fill the device by themselves: one workgroup per tile
        // (streaming loads and stores where whole lines move), spread over
        // the side streams so that one launch's tail overlaps the next one's
        // start; the server's stream waits for them before the read-outs
        if (ns) {
            for (size_t i = 0; i < solo.size(); ++i) {
                const BatchPass *P = solo[i];
                hipStream_t st = s->side[i % ns];
                if (s->dt == QS_C64)
                    launch_tile_f32(P->t, P->ntiles, s->log_r, s->log_nt, st);
                else
                    launch_tile_f64(P->t, P->ntiles, s->log_r, s->log_nt, st);
            }
            for (int i = 0; i < ns; ++i) {
                hipchk(hipEventRecord(s->join_ev[i], s->side[i]), "hipEventRecord");
                hipchk(hipStreamWaitEvent(s->stream, s->join_ev[i], 0), "hipStreamWaitEvent");
            }
        }
        for (int64_t id : step.finishing) {
            SReq &r = s->reqs.at(id);
            double *out = reinterpret_cast<double *>(s->d_bytes + r.res_off);
            launch_zsum(r.state, s->dt, r.n, s->d_zwork, out, s->stream);
            if (!r.samples.empty())
                launch_gather(r.state, s->dt, reinterpret_cast<const uint64_t *>(s->d_bytes + r.samp_off),
                              (int64_t)r.samples.size(), out + r.n + 1, s->stream);
            hipchk(hipMemcpyAsync(s->h_res + (size_t)r.slot * s->res_stride, out, r.res_len, hipMemcpyDeviceToHost,
                                  s->stream),
                   "hipMemcpyAsync(results)");
        }
        hipchk(hipEventRecord(step.ev, s->stream), "hipEventRecord");
        ++s->steps_pending;
        if (n_running)
            *n_running = running;
    });
}

qs_status qs_server_step_wait(qs_server *s, int64_t *ids, int cap, int *n_done)
{
    return guard([&] {
        if (!s)
            fail(QS_ERR_ARG, "server is NULL");
        int w = 0;
        if (s->steps_pending > 0) {
            SStep &step = s->steps[s->step_head];
            hipchk(hipEventSynchronize(step.ev), "hipEventSynchronize");
            s->step_head = (s->step_head + 1) % MAX_STEPS_IN_FLIGHT;
            --s->steps_pending;
            for (int64_t id : step.finishing) {
                SReq &r = s->reqs.at(id);
                const double *h = s->h_res + (size_t)r.slot * s->res_stride;
                r.res.assign(h, h + r.res_len / sizeof(double));
                r.done = true;
                s->free_slots.push_back(r.slot);
                r.slot = -1;
                s->active.erase(std::find(s->active.begin(), s->active.end(), id));
                if (ids && w < cap)
                    ids[w] = id;
                ++w;
            }
            step.finishing.clear();
        }
        if (n_done)
            *n_done = w;
    });
}

qs_status qs_server_result(qs_server *s, int64_t id, double *z, double *amps, double *norm)
{
    return guard([&] {
        if (!s)
            fail(QS_ERR_ARG, "server is NULL");
        auto it = s->reqs.find(id);
        if (it == s->reqs.end() || !it->second.done)
            fail(QS_ERR_STATE, "request unknown or not completed");
        const SReq &r = it->second;
        const double nrm = r.res[0];
        if (norm)
            *norm = nrm;
        if (z)
            for (int q = 0; q < r.n; ++q)
                z[q] = nrm - 2.0 * r.res[1 + q];
        if (amps)
            for (size_t i = 0; i < 2 * r.samples.size(); ++i)
                amps[i] = r.res[r.n + 1 + i];
    });
}

qs_status qs_server_release(qs_server *s, int64_t id)
{
    return guard([&] {
        if (!s)
            fail(QS_ERR_ARG, "server is NULL");
        auto it = s->reqs.find(id);
        if (it == s->reqs.end())
            fail(QS_ERR_ARG, "unknown request");
        SReq &r = it->second;
        if (!r.done)
            fail(QS_ERR_STATE, "request still running");
        s->bytes_alloc.release(r.ops_off, r.ops_len);
        s->bytes_alloc.release(r.samp_off, r.samp_len);
        s->bytes_alloc.release(r.res_off, r.res_len);
        s->pass_alloc.release(r.pass_off, r.np);
        s->resident -= r.bytes;
        s->reqs.erase(it);
    });
}

}  // extern "C"
