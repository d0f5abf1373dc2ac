// C boundary (include/qsim.h): state handles, the program executor and the
// read-out glue.  Every entry point converts internal errors into a status
// code and a per-thread message.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.h"
#include "kernels.h"

using namespace qsim;

struct qs_state {
    int n = 0;
    qs_dtype dt = QS_C128;
    void *buf = nullptr;
    bool owns = false;
    size_t bytes = 0;
    hipStream_t stream = nullptr;
    int dev = 0;
    std::vector<int> sigma;
    double *d_work = nullptr;      // read-out partials and results
    size_t work_doubles = 0;
    uint64_t *d_idx = nullptr;     // gather indices
    double *d_amp = nullptr;       // gathered amplitudes
    int64_t idx_cap = 0;
    qsim::TileOp *d_ops = nullptr; // operation tables of qs_run_circuit (device)
    qsim::TileOp *h_ops = nullptr; // their pinned host staging
    size_t ops_cap = 0;
};

namespace qsim {

[[noreturn]] void fail(qs_status code, const std::string &msg) { throw Error{code, msg}; }

namespace {
thread_local std::string g_err;
}

void set_last_error(const std::string &msg) { g_err = msg; }

}  // namespace qsim

namespace {

template <typename F> qs_status guard(F &&f)
{
    try {
        f();
        g_err.clear();
        return QS_OK;
    } catch (const Error &e) {
        g_err = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        g_err = "host allocation failed";
        return QS_ERR_OOM;
    } catch (const std::exception &e) {
        g_err = e.what();
        return QS_ERR_ARG;
    } catch (...) {
        g_err = "unknown error";
        return QS_ERR_ARG;
    }
}

void hipchk(hipError_t e, const char *what)
{
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(e == hipErrorOutOfMemory ? QS_ERR_OOM : QS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
    }
}

size_t elem_bytes(qs_dtype dt) { return dt == QS_C64 ? 8 : 16; }

void need(bool cond, const char *msg)
{
    if (!cond)
        fail(QS_ERR_ARG, msg);
}

// ---------------------------------------------------------------------------
// launch profiling: HIP events recorded on the launching stream around each
// launch, resolved when read

enum ProfClass { P_TILE, P_U, P_CU, P_CX, P_CZ, P_MOVE, P_BASIS, P_ZSUM, P_GATHER, P_FID, P_ZFOLD, P_NCLASS };
const char *const PROF_NAMES[P_NCLASS] = {"tile_pass", "plain_u", "plain_cu", "plain_cx", "plain_cz",
                                          "move_involution", "set_basis", "zsum", "gather", "fidelity", "zfold"};

struct ProfRec {
    int cls;
    double bytes;
    hipEvent_t a, b;
};

std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_recs;
std::vector<hipEvent_t> g_pool;

hipEvent_t pool_event()
{
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess)
        fail(QS_ERR_HIP, "hipEventCreate");
    return e;
}

template <typename F> void timed(hipStream_t st, int cls, double bytes, F &&f)
{
    if (!g_prof_on) {
        f();
        return;
    }
    std::lock_guard<std::mutex> lk(g_prof_mu);
    hipEvent_t a = pool_event(), b = pool_event();
    if (hipEventRecord(a, st) != hipSuccess)
        fail(QS_ERR_HIP, "hipEventRecord");
    f();
    if (hipEventRecord(b, st) != hipSuccess)
        fail(QS_ERR_HIP, "hipEventRecord");
    g_recs.push_back(ProfRec{cls, bytes, a, b});
}

int gate_class(int kind)
{
    switch (kind) {
    case QS_GATE_U: return P_U;
    case QS_GATE_CU: return P_CU;
    case QS_GATE_CX: return P_CX;
    default: return P_CZ;
    }
}

// algorithmic bytes of one plain gate: every amplitude it must read and write
double gate_bytes(int kind, int n, size_t eb)
{
    const double N = std::ldexp(1.0, n);
    switch (kind) {
    case QS_GATE_U: return 2 * N * eb;
    case QS_GATE_CU:
    case QS_GATE_CX: return N * eb;
    default: return 0.5 * N * eb;
    }
}

void check_perm(const int *sigma, int n)
{
    need(sigma != nullptr, "sigma is NULL");
    std::vector<char> seen(n, 0);
    for (int q = 0; q < n; ++q) {
        need(sigma[q] >= 0 && sigma[q] < n && !seen[sigma[q]], "sigma is not a permutation of 0..n-1");
        seen[sigma[q]] = 1;
    }
}

void check_gate(const qs_gate &g, int n)
{
    need(g.kind >= QS_GATE_U && g.kind <= QS_GATE_CU, "unknown gate kind");
    need(g.q0 >= 0 && g.q0 < n, "gate qubit out of range");
    if (g.kind != QS_GATE_U)
        need(g.q1 >= 0 && g.q1 < n && g.q1 != g.q0, "two-qubit gate needs two distinct qubits in range");
}

void ensure_work(qs_state *s, size_t doubles)
{
    if (s->work_doubles >= doubles)
        return;
    if (s->d_work)
        hipchk(hipFree(s->d_work), "hipFree");
    s->d_work = nullptr;
    s->work_doubles = 0;
    hipchk(hipMalloc(&s->d_work, doubles * sizeof(double)), "hipMalloc(read-out workspace)");
    s->work_doubles = doubles;
}

void ensure_gather(qs_state *s, int64_t count)
{
    if (s->idx_cap >= count)
        return;
    if (s->d_idx)
        hipchk(hipFree(s->d_idx), "hipFree");
    if (s->d_amp)
        hipchk(hipFree(s->d_amp), "hipFree");
    s->d_idx = nullptr;
    s->d_amp = nullptr;
    s->idx_cap = 0;
    hipchk(hipMalloc(&s->d_idx, count * sizeof(uint64_t)), "hipMalloc(gather)");
    hipchk(hipMalloc(&s->d_amp, count * 2 * sizeof(double)), "hipMalloc(gather)");
    s->idx_cap = count;
}

uint64_t phys_index(uint64_t i, const std::vector<int> &sigma)
{
    uint64_t j = 0;
    for (size_t q = 0; q < sigma.size(); ++q)
        if ((i >> q) & 1)
            j |= 1ull << sigma[q];
    return j;
}

// Apply the position map pi (amplitude at x moves to the index whose bit
// pi[p] is bit p of x) as at most two in-place involutions: along each cycle
// c_0 -> c_1 -> ... -> c_{L-1} of pi, first c_i -> c_{-i}, then c_i -> c_{1-i}
// (indices mod L); the composition sends c_i to c_{i+1}.
// Physical position p of the state moves to pi[p] (PermuteQubits, Section 2).
//
// The position map's cycles are grouped so that each group's positions, plus
// the lowest positions (so that every load and store moves 128-byte runs), fit
// a tile.  A group is one tile pass without gates that writes each tile back
// with its bits permuted: the tile is closed under the map, so the move stays
// inside the tile, in place, and every amplitude is read and written once.
// Cycles too long for a tile go through two in-place involutions instead.
void apply_position_map(qs_state *s, const std::vector<int> &pi)
{
    const int n = s->n;
    const int esize = elem_bytes(s->dt);
    int low = 0;
    while ((esize << low) < DIRECT_RUN_BYTES)
        ++low;
    const int max_k = std::min(n, esize == 16 ? 12 : 13);  // tiles of at most 64 KiB
    std::vector<std::vector<int>> cycles;
    std::vector<char> seen(n, 0);
    size_t longest = 0;
    for (int p = 0; p < n; ++p) {
        if (seen[p])
            continue;
        std::vector<int> cyc;
        for (int x = p; !seen[x]; x = pi[x]) {
            seen[x] = 1;
            cyc.push_back(x);
        }
        if (cyc.size() > 1) {
            longest = std::max(longest, cyc.size());
            cycles.push_back(cyc);
        }
    }
    if (cycles.empty())
        return;
    auto tile_bits = [&](const std::vector<int> &moved) {
        std::vector<char> in(n, 0);
        for (int p : moved)
            in[p] = 1;
        int k = (int)moved.size();
        for (int p = 0; p < n && (p < low || k < MIN_TILE_BITS); ++p)
            if (!in[p]) {
                in[p] = 1;
                ++k;
            }
        return k;
    };
    if (n >= MIN_TILE_BITS && (int)longest + low <= max_k) {
        std::vector<std::vector<int>> groups;
        for (const auto &c : cycles) {
            bool placed = false;
            for (auto &g : groups) {
                std::vector<int> t = g;
                t.insert(t.end(), c.begin(), c.end());
                if (tile_bits(t) <= max_k) {
                    g = t;
                    placed = true;
                    break;
                }
            }
            if (!placed)
                groups.push_back(c);
        }
        for (const auto &g : groups) {
            std::vector<char> in(n, 0);
            for (int p : g)
                in[p] = 1;
            std::vector<int> pos = g;
            for (int p = 0; p < n && (p < low || (int)pos.size() < MIN_TILE_BITS); ++p)
                if (!in[p]) {
                    in[p] = 1;
                    pos.push_back(p);
                }
            std::sort(pos.begin(), pos.end());
            const int k = (int)pos.size();
            int log_r = 0, log_nt = 0;
            tile_shape(k, s->dt, 0, &log_r, &log_nt);
            TileArgs a{};
            tile_args_for_positions(pos, log_nt, log_r, a);
            std::vector<int> tb(n, -1);
            for (int b = 0; b < k; ++b)
                tb[pos[b]] = b;
            // this group's cycles only; the padding positions stay (another
            // group may move them in its own pass)
            std::vector<char> mine(n, 0);
            for (int p : g)
                mine[p] = 1;
            for (int b = 0; b < k; ++b)
                a.sperm[b] = (uint8_t)(mine[pos[b]] ? tb[pi[pos[b]]] : b);
            // permuted store; the tile holds the lowest positions, so every
            // load and store moves whole lines (streaming access)
            a.io = 4u | 8u;
            a.state = s->buf;
            a.ops = nullptr;
            a.n_ops = 0;
            a.n_hi = n - k;
            const uint64_t tiles = 1ull << (n - k);
            timed(s->stream, P_MOVE, 2.0 * (double)s->bytes, [&] {
                if (s->dt == QS_C64)
                    launch_tile_f32(a, tiles, log_r, log_nt, s->stream);
                else
                    launch_tile_f64(a, tiles, log_r, log_nt, s->stream);
            });
        }
        return;
    }
    std::vector<int> r1(n), r2(n);
    for (int p = 0; p < n; ++p)
        r1[p] = r2[p] = p;
    for (const auto &cyc : cycles) {
        const int L = (int)cyc.size();
        for (int i = 0; i < L; ++i) {
            r1[cyc[i]] = cyc[((-i) % L + L) % L];
            r2[cyc[i]] = cyc[((1 - i) % L + L) % L];
        }
    }
    for (const std::vector<int> *r : {&r1, &r2}) {
        int pairs = 0;
        for (int p = 0; p < n; ++p)
            pairs += (*r)[p] > p;
        if (pairs == 0)
            continue;
        const double bytes = 2.0 * (1.0 - std::ldexp(1.0, -pairs)) * std::ldexp(1.0, n) * elem_bytes(s->dt);
        timed(s->stream, P_MOVE, bytes, [&] { launch_involution(s->buf, s->dt, n, *r, s->stream); });
    }
}

void upload_ops(Program &p)
{
    int dev = 0;
    hipchk(hipGetDevice(&dev), "hipGetDevice");
    if (p.d_ops && p.dev == dev)
        return;
    if (p.ops.empty())
        return;
    if (p.d_ops) {
        int cur = dev;
        hipchk(hipSetDevice(p.dev), "hipSetDevice");
        (void)hipFree(p.d_ops);
        hipchk(hipSetDevice(cur), "hipSetDevice");
        p.d_ops = nullptr;
    }
    hipchk(hipMalloc(&p.d_ops, p.ops.size() * sizeof(TileOp)), "hipMalloc(tile ops)");
    hipchk(hipMemcpy(p.d_ops, p.ops.data(), p.ops.size() * sizeof(TileOp), hipMemcpyHostToDevice),
           "hipMemcpy(tile ops)");
    p.dev = dev;
}

// Enqueue launches [a, b) of p; tile operations are read from d_ops.  A
// program run from |0...0> (QS_OPT_FROM_ZERO) has its first tile pass start
// from the basis state in registers; any other first launch gets the state
// set first.
void launch_range(qs_state *s, const Program &p, size_t a_idx, size_t b_idx, const TileOp *d_ops,
                  double *zparts = nullptr)
{
    const bool from_zero = (p.opts.flags & QS_OPT_FROM_ZERO) != 0;
    for (size_t li = a_idx; li < b_idx; ++li) {
        const Launch &L = p.launches[li];
        const bool basis = from_zero && li == 0;
        if (basis && L.type != L_TILE)
            timed(s->stream, P_BASIS, (double)s->bytes, [&] { launch_set_basis(s->buf, s->dt, s->n, 0, s->stream); });
        switch (L.type) {
        case L_PLAIN:
            timed(s->stream, gate_class(L.gate.kind), gate_bytes(L.gate.kind, s->n, elem_bytes(s->dt)),
                  [&] { launch_plain_gate(s->buf, s->dt, s->n, L.gate, s->stream); });
            break;
        case L_MOVE:
            apply_position_map(s, L.pi);
            break;
        case L_TILE: {
            TileArgs a{};
            tile_args_from_launch(L, a);
            a.state = s->buf;
            a.ops = d_ops + L.op_begin;
            a.n_hi = s->n - L.k;
            if (basis)
                a.io |= IO_BASIS;
            const uint64_t tiles = 1ull << (s->n - L.k);
            // a pass from the basis state reads nothing
            timed(s->stream, P_TILE, (basis ? 1.0 : 2.0) * (double)s->bytes, [&] {
                if (zparts && s->dt == QS_C64)
                    launch_tile_f32_z(a, tiles, L.log_r, L.log_nt, zparts, s->stream);
                else if (zparts)
                    launch_tile_f64_z(a, tiles, L.log_r, L.log_nt, zparts, s->stream);
                else if (s->dt == QS_C64)
                    launch_tile_f32(a, tiles, L.log_r, L.log_nt, s->stream);
                else
                    launch_tile_f64(a, tiles, L.log_r, L.log_nt, s->stream);
            });
            break;
        }
        }
    }
}

void check_program_fits(const qs_state *s, const Program &p)
{
    need(s->n == p.n, "program compiled for a different qubit count");
    need(s->dt == p.dt, "program compiled for a different amplitude type");
    if (s->sigma != p.sigma0)
        fail(QS_ERR_STATE, "state placement differs from the program's starting placement");
}

// A program with no launch run from |0...0> still sets the state.
void finish_empty(qs_state *s, const Program &p)
{
    if ((p.opts.flags & QS_OPT_FROM_ZERO) && p.launches.empty())
        timed(s->stream, P_BASIS, (double)s->bytes, [&] { launch_set_basis(s->buf, s->dt, s->n, 0, s->stream); });
}

void run_launches(qs_state *s, Program &p)
{
    check_program_fits(s, p);
    upload_ops(p);
    launch_range(s, p, 0, p.launches.size(), p.d_ops);
    finish_empty(s, p);
    s->sigma = p.sigma_final;
}

// Operation tables of qs_run_circuit: a device buffer and its pinned staging,
// kept with the state and grown on demand (every call ends synchronised, so
// the next one may overwrite them).
void ensure_op_buffers(qs_state *s, size_t n_ops)
{
    if (n_ops <= s->ops_cap)
        return;
    if (s->d_ops)
        (void)hipFree(s->d_ops);
    if (s->h_ops)
        (void)hipHostFree(s->h_ops);
    s->d_ops = nullptr;
    s->h_ops = nullptr;
    s->ops_cap = 0;
    hipchk(hipMalloc(&s->d_ops, n_ops * sizeof(TileOp)), "hipMalloc(tile ops)");
    hipchk(hipHostMalloc(&s->h_ops, n_ops * sizeof(TileOp), hipHostMallocDefault), "hipHostMalloc(tile ops)");
    s->ops_cap = n_ops;
}

qs_run_opts default_opts()
{
    qs_run_opts o{};
    o.form = QS_FORM_PASS;
    o.k_tile = 12;
    o.max_swaps = 1;
    o.pinned = 0;
    o.perm_exec = QS_PERM_MOVE;
    return o;
}

}  // namespace

namespace qsim {

void check_program_on(const qs_state *s, const Program &p)
{
    need(s != nullptr, "state is NULL");
    check_program_fits(s, p);
}

void run_program_with_ops(qs_state *s, const Program &p, const TileOp *d_ops)
{
    check_program_on(s, p);
    launch_range(s, p, 0, p.launches.size(), d_ops);
    finish_empty(s, p);
    s->sigma = p.sigma_final;
}

void *state_stream(const qs_state *s) { return s->stream; }
int state_device(const qs_state *s) { return s->dev; }

qs_status guarded(const std::function<void()> &f) { return guard(f); }

}  // namespace qsim

extern "C" {

const char *qs_last_error(void) { return g_err.c_str(); }

qs_status qs_device_info(int *cu_count, int *lds_bytes, size_t *hbm_bytes, char *name, int name_len)
{
    return guard([&] {
        int dev = 0;
        hipchk(hipGetDevice(&dev), "hipGetDevice");
        hipDeviceProp_t prop;
        hipchk(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
        if (cu_count)
            *cu_count = prop.multiProcessorCount;
        if (lds_bytes)
            *lds_bytes = (int)prop.maxSharedMemoryPerMultiProcessor;
        if (hbm_bytes)
            *hbm_bytes = prop.totalGlobalMem;
        if (name && name_len > 0) {
            std::string nm = std::string(prop.name) + " " + prop.gcnArchName;
            std::strncpy(name, nm.c_str(), (size_t)name_len - 1);
            name[name_len - 1] = 0;
        }
    });
}

qs_status qs_state_create(int n, qs_dtype dt, void *device_buf, size_t buf_bytes, void *stream, qs_state **out)
{
    return guard([&] {
        need(out != nullptr, "out is NULL");
        *out = nullptr;
        need(n >= 1 && n <= MAX_QUBITS, "n must be in [1, 34]");
        need(dt == QS_C64 || dt == QS_C128, "unknown dtype");
        const size_t bytes = elem_bytes(dt) << n;
        auto *s = new qs_state();
        try {
            s->n = n;
            s->dt = dt;
            s->stream = reinterpret_cast<hipStream_t>(stream);
            hipchk(hipGetDevice(&s->dev), "hipGetDevice");
            s->sigma.resize(n);
            for (int q = 0; q < n; ++q)
                s->sigma[q] = q;
            if (device_buf) {
                need(buf_bytes >= bytes, "device buffer smaller than 2^n amplitudes");
                need(reinterpret_cast<uintptr_t>(device_buf) % 16 == 0, "device buffer must be 16-byte aligned");
                s->buf = device_buf;
                s->owns = false;
            } else {
                hipchk(hipMalloc(&s->buf, bytes), "hipMalloc(state)");
                s->owns = true;
            }
            s->bytes = bytes;
            launch_set_basis(s->buf, dt, n, 0, s->stream);
        } catch (...) {
            if (s->owns && s->buf)
                (void)hipFree(s->buf);
            delete s;
            throw;
        }
        *out = s;
    });
}

qs_status qs_state_destroy(qs_state *s)
{
    return guard([&] {
        if (!s)
            return;
        (void)hipStreamSynchronize(s->stream);
        if (s->owns && s->buf)
            (void)hipFree(s->buf);
        if (s->d_work)
            (void)hipFree(s->d_work);
        if (s->d_idx)
            (void)hipFree(s->d_idx);
        if (s->d_amp)
            (void)hipFree(s->d_amp);
        if (s->d_ops)
            (void)hipFree(s->d_ops);
        if (s->h_ops)
            (void)hipHostFree(s->h_ops);
        delete s;
    });
}

qs_status qs_state_set_stream(qs_state *s, void *stream)
{
    return guard([&] {
        need(s != nullptr, "state is NULL");
        s->stream = reinterpret_cast<hipStream_t>(stream);
    });
}

qs_status qs_state_info(const qs_state *s, int *n, int *dtype, void **device_buf)
{
    return guard([&] {
        need(s != nullptr, "state is NULL");
        if (n)
            *n = s->n;
        if (dtype)
            *dtype = (int)s->dt;
        if (device_buf)
            *device_buf = s->buf;
    });
}

qs_status qs_state_set_basis(qs_state *s, uint64_t x)
{
    return guard([&] {
        need(s != nullptr, "state is NULL");
        need(s->n == 64 || x < (1ull << s->n), "basis index out of range");
        for (int q = 0; q < s->n; ++q)
            s->sigma[q] = q;
        timed(s->stream, P_BASIS, (double)s->bytes, [&] { launch_set_basis(s->buf, s->dt, s->n, x, s->stream); });
    });
}

qs_status qs_get_permutation(const qs_state *s, int *sigma)
{
    return guard([&] {
        need(s != nullptr && sigma != nullptr, "NULL argument");
        std::copy(s->sigma.begin(), s->sigma.end(), sigma);
    });
}

qs_status qs_apply_gate(qs_state *s, const qs_gate *g) { return qs_apply_gates(s, g, 1); }

qs_status qs_apply_gates(qs_state *s, const qs_gate *g, int64_t n_gates)
{
    return guard([&] {
        need(s != nullptr && (g != nullptr || n_gates == 0), "NULL argument");
        need(n_gates >= 0, "negative gate count");
        for (int64_t i = 0; i < n_gates; ++i)
            check_gate(g[i], s->n);
        for (int64_t i = 0; i < n_gates; ++i) {
            qs_gate p = g[i];
            p.q0 = s->sigma[g[i].q0];
            p.q1 = g[i].kind == QS_GATE_U ? -1 : s->sigma[g[i].q1];
            timed(s->stream, gate_class(p.kind), gate_bytes(p.kind, s->n, elem_bytes(s->dt)),
                  [&] { launch_plain_gate(s->buf, s->dt, s->n, p, s->stream); });
        }
    });
}

qs_status qs_permute_qubits(qs_state *s, const int *sigma_new)
{
    return guard([&] {
        need(s != nullptr, "state is NULL");
        check_perm(sigma_new, s->n);
        std::vector<int> pi(s->n);
        for (int q = 0; q < s->n; ++q)
            pi[s->sigma[q]] = sigma_new[q];
        apply_position_map(s, pi);
        s->sigma.assign(sigma_new, sigma_new + s->n);
    });
}

namespace {
void check_costs(const qs_pass_costs &c)
{
    const double v[] = {c.tile_pass, c.in_pass[0], c.in_pass[1], c.in_pass[2], c.move,
                        c.plain[0], c.plain[1], c.plain[2], c.plain[3]};
    for (double x : v)
        need(std::isfinite(x) && x >= 0.0, "pass costs must be finite and non-negative");
}

qs_status compile_entry(const qs_gate *gates, int64_t n_gates, int n, qs_dtype dt, const int *sigma0,
                        const qs_run_opts *opts, const qs_pass_costs *costs, qs_program **out)
{
    return guard([&] {
        need(out != nullptr, "out is NULL");
        *out = nullptr;
        need(gates != nullptr || n_gates == 0, "gates is NULL");
        need(n_gates >= 0 && n_gates < (1ll << 30), "gate count out of range");
        need(n >= 1 && n <= MAX_COMPILE_QUBITS, "n must be in [1, 63]");
        need(dt == QS_C64 || dt == QS_C128, "unknown dtype");
        if (sigma0)
            check_perm(sigma0, n);
        for (int64_t i = 0; i < n_gates; ++i)
            check_gate(gates[i], n);
        qs_run_opts o = opts ? *opts : default_opts();
        if (o.form == QS_FORM_PASS)
            need(o.k_tile >= 1, "k_tile must be >= 1");
        if (costs)
            check_costs(*costs);
        auto *p = new qs_program();
        try {
            compile_program(gates, n_gates, n, dt, sigma0, o, p->p, {}, costs);
        } catch (...) {
            delete p;
            throw;
        }
        *out = p;
    });
}
}  // namespace

qs_status qs_compile(const qs_gate *gates, int64_t n_gates, int n, qs_dtype dt, const int *sigma0,
                     const qs_run_opts *opts, qs_program **out)
{
    return compile_entry(gates, n_gates, n, dt, sigma0, opts, nullptr, out);
}

qs_status qs_compile_costed(const qs_gate *gates, int64_t n_gates, int n, qs_dtype dt, const int *sigma0,
                            const qs_run_opts *opts, const qs_pass_costs *costs, qs_program **out)
{
    if (!costs)
        return guard([&] { need(false, "costs is NULL"); });
    return compile_entry(gates, n_gates, n, dt, sigma0, opts, costs, out);
}

qs_status qs_program_destroy(qs_program *p)
{
    return guard([&] {
        if (!p)
            return;
        if (p->p.d_ops) {
            int cur = 0;
            (void)hipGetDevice(&cur);
            (void)hipSetDevice(p->p.dev);
            (void)hipDeviceSynchronize();
            (void)hipFree(p->p.d_ops);
            (void)hipSetDevice(cur);
        }
        delete p;
    });
}

qs_status qs_program_get_stats(const qs_program *p, qs_program_stats *out)
{
    return guard([&] {
        need(p != nullptr && out != nullptr, "NULL argument");
        *out = p->p.stats;
    });
}

qs_status qs_program_op_counts(const qs_program *p, double *out, int cap)
{
    return guard([&] {
        need(p != nullptr && (out != nullptr || cap <= 0), "NULL argument");
        double c[QS_OPC_COUNT] = {};
        const Program &P = p->p;
        for (const Launch &L : P.launches) {
            if (L.type == L_TILE) {
                c[QS_OPC_TILE_PASS] += 1;
                for (int i = 0; i < L.op_count; ++i) {
                    const TileOp &o = P.ops[L.op_begin + i];
                    if (o.kind == OP_REMAP) {
                        c[QS_OPC_REMAP] += 1;
                        c[QS_OPC_REMAP_WAVE] += (o.aux & REMAP_WAVE_LOCAL) ? 1 : 0;
                        continue;
                    }
                    if (o.kind == OP_SHEAR2) {
                        c[QS_OPC_SHEAR] += 2;
                        continue;
                    }
                    if (o.kind == OP_LSWAP) {
                        c[QS_OPC_LSWAP] += 1;
                        continue;
                    }
                    if (o.kind == OP_LANE) {
                        c[QS_OPC_LANE] += 1;
                        continue;
                    }
                    const double w = std::ldexp(1.0, -__builtin_popcountll(o.hmask));
                    const bool ctrl = (o.rmask | o.lmask) != 0;
                    c[QS_OPC_DISPATCH] += 1.0 - w;
                    switch (o.kind) {
                    case OP_U:
                        c[ctrl ? QS_OPC_U_CTRL : QS_OPC_U] += w;
                        break;
                    case OP_X:
                        if (!ctrl)
                            c[QS_OPC_DISPATCH] += w;
                        else
                            c[o.lmask ? QS_OPC_X_LANE : QS_OPC_X_REG] += w;
                        break;
                    case OP_NEG:
                        c[QS_OPC_NEG] += w;
                        break;
                    case OP_SHEAR:
                        c[QS_OPC_SHEAR] += w;
                        break;
                    case OP_PHASE:
                        c[QS_OPC_PHASE] += w;
                        break;
                    default:
                        c[QS_OPC_DIAG] += w;
                        break;
                    }
                }
            } else if (L.type == L_PLAIN) {
                switch (L.gate.kind) {
                case QS_GATE_U: c[QS_OPC_PLAIN_U] += 1; break;
                case QS_GATE_CU: c[QS_OPC_PLAIN_CU] += 1; break;
                case QS_GATE_CX: c[QS_OPC_PLAIN_CX] += 1; break;
                default: c[QS_OPC_PLAIN_CZ] += 1; break;
                }
            } else {
                c[QS_OPC_MOVE] += 1;
                int moved = 0;
                for (size_t q = 0; q < L.pi.size(); ++q)
                    moved += L.pi[q] != (int)q;
                // an exchange of m positions leaves the amplitudes whose moved
                // bits are all equal in place
                c[QS_OPC_MOVE_FRACTION] += moved ? 1.0 - std::ldexp(1.0, -(moved / 2)) : 0.0;
            }
        }
        for (int i = 0; i < cap && i < QS_OPC_COUNT; ++i)
            out[i] = c[i];
    });
}

qs_status qs_program_instructions(const qs_program *p, int32_t *buf, int64_t cap, int64_t *len)
{
    return guard([&] {
        need(p != nullptr && len != nullptr, "NULL argument");
        int64_t w = 0;
        auto put = [&](int32_t x) {
            if (buf && w < cap)
                buf[w] = x;
            ++w;
        };
        for (const Instr &I : p->p.instrs) {
            put(I.type);
            if (I.type == 1)
                for (int x : I.sigma)
                    put(x);
            else
                put(I.gate);
        }
        *len = w;
    });
}

qs_status qs_run_program(qs_state *s, const qs_program *p)
{
    return guard([&] {
        need(s != nullptr && p != nullptr, "NULL argument");
        run_launches(s, const_cast<qs_program *>(p)->p);
    });
}

static void zsum(qs_state *s, std::vector<double> &res);

// Compile and run.  In the pass form the launches of each segment are
// enqueued as soon as the pass has fixed it, so the device works on the first
// segments while the host is still choosing later permutations.  With ez the
// last launch is held back until the program is complete: when it is a tile
// pass it also writes per-tile probability sums, folded into the sums of
// qs_expect_z (no read-out pass over the state); otherwise the read-out pass
// runs after it.  ez receives <Z_q> (host, n doubles).
namespace {
// Launches [from, end) of a complete program, then <Z_q> into ez.  When the
// last tile pass moves whole lines and every launch after it is a CNOT or CZ
// on its own, that pass writes its per-tile sums: a CZ leaves every bit's
// probability alone and a CNOT makes its target bit the XOR of target and
// control, so each final bit is an XOR of bits after the pass, folded from
// those sums (when at most one of the XORed bits is a tile bit).  Otherwise
// the read-out pass runs after the last launch.
void fused_expect_z(qs_state *s, const Program &p, const TileOp *d_ops, size_t from, double *ez)
{
    const size_t end = p.launches.size();
    size_t lt = end;
    for (size_t li = end; li-- > from;)
        if (p.launches[li].type == L_TILE) {
            lt = li;
            break;
        }
    bool fold = lt < end && (p.launches[lt].io & 8u) && !(p.launches[lt].io & 4u);
    // bit p after the program = XOR of the bits in mask[p] after the pass
    std::vector<uint64_t> mask(s->n);
    for (int q = 0; q < s->n; ++q)
        mask[q] = 1ull << q;
    for (size_t li = lt + 1; fold && li < end; ++li) {
        const Launch &L = p.launches[li];
        if (L.type != L_PLAIN || (L.gate.kind != QS_GATE_CX && L.gate.kind != QS_GATE_CZ))
            fold = false;
        else if (L.gate.kind == QS_GATE_CX)
            mask[L.gate.q1] ^= mask[L.gate.q0];
    }
    ZFoldMap m{};
    if (fold) {
        const Launch &L = p.launches[lt];
        std::vector<int> layout(s->n, 0), rank(s->n, -1);
        for (int q = 0; q < L.log_r; ++q)
            layout[L.st_reg[q]] = 1 + q;
        for (int i = 0; i < L.log_nt; ++i)
            layout[L.st_lane[i]] = 1 + L.log_r + i;
        for (int pos = 0, r = 0; pos < s->n; ++pos)
            if (!layout[pos])
                rank[pos] = r++;
        for (int pos = 0; pos < s->n && fold; ++pos) {
            m.v[pos] = 0;
            m.rm[pos] = 0;
            for (int b = 0; b < s->n; ++b) {
                if (!((mask[pos] >> b) & 1u))
                    continue;
                if (layout[b]) {
                    fold = m.v[pos] == 0;  // at most one tile bit
                    m.v[pos] = layout[b];
                } else {
                    m.rm[pos] |= 1ull << rank[b];
                }
            }
        }
    }
    std::vector<double> r(s->n + 1);
    if (fold) {
        const Launch &L = p.launches[lt];
        const int nv = 1 + L.log_r + L.log_nt;
        const uint64_t tiles = 1ull << (s->n - L.k);
        const size_t fw = zfold_work_doubles(tiles, s->n);
        ensure_work(s, (size_t)tiles * nv + fw + (size_t)s->n + 1);
        double *parts = s->d_work, *fwork = parts + (size_t)tiles * nv, *outd = fwork + fw;
        launch_range(s, p, from, lt, d_ops);
        launch_range(s, p, lt, lt + 1, d_ops, parts);
        launch_range(s, p, lt + 1, end, d_ops);
        timed(s->stream, P_ZFOLD, (double)tiles * nv * sizeof(double),
              [&] { launch_zfold(parts, tiles, nv, s->n, m, fwork, outd, s->stream); });
        hipchk(hipMemcpyAsync(r.data(), outd, (s->n + 1) * sizeof(double), hipMemcpyDeviceToHost, s->stream),
               "hipMemcpyAsync");
        hipchk(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    } else {
        launch_range(s, p, from, end, d_ops);
        zsum(s, r);
    }
    for (int q = 0; q < s->n; ++q)
        ez[q] = r[0] - 2.0 * r[1 + p.sigma_final[q]];
}

qs_status run_circuit_entry(qs_state *s, const qs_gate *gates, int64_t n_gates, const qs_run_opts *opts,
                            const qs_pass_costs *costs, double *ez = nullptr)
{
    return guard([&] {
        need(s != nullptr, "state is NULL");
        need(n_gates >= 0 && (n_gates == 0 || gates != nullptr), "bad arguments");
        const qs_run_opts o = opts ? *opts : default_opts();
        if (costs)
            check_costs(*costs);
        Program p;
        // the plain form's program table, freed on every way out (after the
        // stream has been synchronised)
        struct FreeOps {
            Program &p;
            ~FreeOps()
            {
                if (p.d_ops)
                    (void)hipFree(p.d_ops);
            }
        } free_ops{p};
        // every gate gives at most its operation, two pending factors applied
        // before it and one re-layout; every segment (at most one per gate)
        // one more re-layout and two lane swaps
        const size_t bound = 7 * (size_t)n_gates + 16;
        if (o.form == QS_FORM_PASS)
            ensure_op_buffers(s, bound);
        size_t launched = 0, uploaded = 0;
        auto progress = [&](Program &pp) {
            if (pp.ops.size() > bound)
                fail(QS_ERR_UNSUPPORTED, "internal: operation table larger than its bound");
            if (pp.ops.size() > uploaded) {
                const size_t cnt = pp.ops.size() - uploaded;
                std::memcpy(s->h_ops + uploaded, pp.ops.data() + uploaded, cnt * sizeof(TileOp));
                hipchk(hipMemcpyAsync(s->d_ops + uploaded, s->h_ops + uploaded, cnt * sizeof(TileOp),
                                      hipMemcpyHostToDevice, s->stream),
                       "hipMemcpyAsync(tile ops)");
                uploaded = pp.ops.size();
            }
            // with ez the newest tile pass and the launches after it wait:
            // that pass may be the one that folds in the read-out
            size_t upto = pp.launches.size();
            if (ez)
                for (size_t li = upto; li-- > launched;)
                    if (pp.launches[li].type == L_TILE) {
                        upto = li;
                        break;
                    }
            if (upto > launched) {
                launch_range(s, pp, launched, upto, s->d_ops);
                launched = upto;
            }
        };
        if (o.form == QS_FORM_PASS) {
            try {
                compile_program(gates, n_gates, s->n, s->dt, s->sigma.data(), o, p, progress, costs);
            } catch (...) {
                // launches already enqueued read the op tables: let them
                // finish before the error is reported (the state then holds a
                // partly applied circuit)
                (void)hipStreamSynchronize(s->stream);
                throw;
            }
            if (ez && launched < p.launches.size()) {
                try {
                    fused_expect_z(s, p, s->d_ops, launched, ez);
                } catch (...) {
                    (void)hipStreamSynchronize(s->stream);
                    throw;
                }
                ez = nullptr;
            }
            finish_empty(s, p);
            s->sigma = p.sigma_final;
        } else {
            compile_program(gates, n_gates, s->n, s->dt, s->sigma.data(), o, p);
            try {
                run_launches(s, p);
            } catch (...) {
                (void)hipStreamSynchronize(s->stream);
                throw;
            }
        }
        if (ez) {
            std::vector<double> r;
            zsum(s, r);
            for (int q = 0; q < s->n; ++q)
                ez[q] = r[0] - 2.0 * r[1 + s->sigma[q]];
        }
        // the tables (and the staging the copies read) are reused next call
        hipchk(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    });
}
}  // namespace

qs_status qs_run_circuit(qs_state *s, const qs_gate *gates, int64_t n_gates, const qs_run_opts *opts)
{
    return run_circuit_entry(s, gates, n_gates, opts, nullptr);
}

qs_status qs_run_circuit_costed(qs_state *s, const qs_gate *gates, int64_t n_gates, const qs_run_opts *opts,
                                const qs_pass_costs *costs)
{
    if (!costs)
        return guard([&] { need(false, "costs is NULL"); });
    return run_circuit_entry(s, gates, n_gates, opts, costs);
}

qs_status qs_run_circuit_expect_z(qs_state *s, const qs_gate *gates, int64_t n_gates, const qs_run_opts *opts,
                                  const qs_pass_costs *costs, double *expect_z)
{
    if (!expect_z)
        return guard([&] { need(false, "expect_z is NULL"); });
    return run_circuit_entry(s, gates, n_gates, opts, costs, expect_z);
}

qs_status qs_synchronize(qs_state *s)
{
    return guard([&] {
        need(s != nullptr, "state is NULL");
        hipchk(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    });
}

qs_status qs_read_amplitudes(qs_state *s, const uint64_t *idx, int64_t count, double *out)
{
    return guard([&] {
        need(s != nullptr, "state is NULL");
        need(count >= 0 && (count == 0 || (idx && out)), "bad arguments");
        if (count == 0)
            return;
        std::vector<uint64_t> phys(count);
        for (int64_t i = 0; i < count; ++i) {
            need(s->n == 64 || idx[i] < (1ull << s->n), "amplitude index out of range");
            phys[i] = phys_index(idx[i], s->sigma);
        }
        ensure_gather(s, count);
        hipchk(hipMemcpyAsync(s->d_idx, phys.data(), count * sizeof(uint64_t), hipMemcpyHostToDevice, s->stream),
               "hipMemcpyAsync");
        timed(s->stream, P_GATHER, (double)count * elem_bytes(s->dt),
              [&] { launch_gather(s->buf, s->dt, s->d_idx, count, s->d_amp, s->stream); });
        hipchk(hipMemcpyAsync(out, s->d_amp, count * 2 * sizeof(double), hipMemcpyDeviceToHost, s->stream),
               "hipMemcpyAsync");
        hipchk(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    });
}

qs_status qs_read_state(qs_state *s, double *out)
{
    return guard([&] {
        need(s != nullptr && out != nullptr, "NULL argument");
        need(s->n <= 30, "qs_read_state is limited to n <= 30");
        const uint64_t N = 1ull << s->n;
        std::vector<unsigned char> raw(s->bytes);
        hipchk(hipMemcpyAsync(raw.data(), s->buf, s->bytes, hipMemcpyDeviceToHost, s->stream), "hipMemcpyAsync");
        hipchk(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
        for (uint64_t i = 0; i < N; ++i) {
            const uint64_t j = phys_index(i, s->sigma);
            if (s->dt == QS_C64) {
                const float *f = reinterpret_cast<const float *>(raw.data());
                out[2 * i] = f[2 * j];
                out[2 * i + 1] = f[2 * j + 1];
            } else {
                const double *d = reinterpret_cast<const double *>(raw.data());
                out[2 * i] = d[2 * j];
                out[2 * i + 1] = d[2 * j + 1];
            }
        }
    });
}

static void zsum(qs_state *s, std::vector<double> &res)
{
    const size_t w = zsum_work_doubles(s->n) + (size_t)s->n + 1;
    ensure_work(s, std::max(w, fid_work_doubles(s->n) + 5));
    double *outd = s->d_work + zsum_work_doubles(s->n);
    timed(s->stream, P_ZSUM, (double)s->bytes, [&] { launch_zsum(s->buf, s->dt, s->n, s->d_work, outd, s->stream); });
    res.resize(s->n + 1);
    hipchk(hipMemcpyAsync(res.data(), outd, (s->n + 1) * sizeof(double), hipMemcpyDeviceToHost, s->stream),
           "hipMemcpyAsync");
    hipchk(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
}

qs_status qs_expect_z(qs_state *s, double *out)
{
    return guard([&] {
        need(s != nullptr && out != nullptr, "NULL argument");
        std::vector<double> r;
        zsum(s, r);
        for (int q = 0; q < s->n; ++q)
            out[q] = r[0] - 2.0 * r[1 + s->sigma[q]];
    });
}

qs_status qs_norm(qs_state *s, double *out)
{
    return guard([&] {
        need(s != nullptr && out != nullptr, "NULL argument");
        std::vector<double> r;
        zsum(s, r);
        *out = r[0];
    });
}

qs_status qs_fidelity(qs_state *a, qs_state *b, double *loss, double *max_abs_diff)
{
    return guard([&] {
        need(a != nullptr && b != nullptr, "NULL state");
        need(a->n == b->n, "states differ in qubit count");
        const int n = a->n;
        std::vector<int> inv_a(n), map_b(n);
        for (int q = 0; q < n; ++q)
            inv_a[a->sigma[q]] = q;
        for (int p = 0; p < n; ++p)
            map_b[p] = b->sigma[inv_a[p]];
        // b's pending work must finish before a's stream reads it
        hipchk(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
        ensure_work(a, std::max(fid_work_doubles(n) + 5, zsum_work_doubles(n) + (size_t)n + 1));
        double *outd = a->d_work + fid_work_doubles(n);
        timed(a->stream, P_FID, (double)(a->bytes + b->bytes),
              [&] { launch_fidelity(a->buf, a->dt, b->buf, b->dt, n, map_b, a->d_work, outd, a->stream); });
        double r[5];
        hipchk(hipMemcpyAsync(r, outd, sizeof r, hipMemcpyDeviceToHost, a->stream), "hipMemcpyAsync");
        hipchk(hipStreamSynchronize(a->stream), "hipStreamSynchronize");
        const double ov = r[0] * r[0] + r[1] * r[1];
        if (loss)
            *loss = 1.0 - ov / (r[2] * r[3]);
        if (max_abs_diff)
            *max_abs_diff = r[4];
    });
}

qs_status qs_profile_enable(int on)
{
    return guard([&] {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        g_prof_on = on != 0;
    });
}

qs_status qs_profile_read(qs_profile_entry *out, int cap, int *n_out)
{
    return guard([&] {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        int64_t cnt[P_NCLASS] = {};
        double ms[P_NCLASS] = {}, by[P_NCLASS] = {};
        for (const ProfRec &r : g_recs) {
            hipchk(hipEventSynchronize(r.b), "hipEventSynchronize");
            float t = 0;
            hipchk(hipEventElapsedTime(&t, r.a, r.b), "hipEventElapsedTime");
            cnt[r.cls] += 1;
            ms[r.cls] += t;
            by[r.cls] += r.bytes;
            g_pool.push_back(r.a);
            g_pool.push_back(r.b);
        }
        g_recs.clear();
        int w = 0;
        for (int c = 0; c < P_NCLASS; ++c) {
            if (cnt[c] == 0)
                continue;
            if (out && w < cap) {
                std::memset(&out[w], 0, sizeof out[w]);
                std::strncpy(out[w].name, PROF_NAMES[c], sizeof out[w].name - 1);
                out[w].launches = cnt[c];
                out[w].total_ms = ms[c];
                out[w].bytes = by[c];
            }
            ++w;
        }
        if (n_out)
            *n_out = w;
    });
}

}  // extern "C"
