// Circuit compiler: dependency DAG with exact commutation, the
// permutation-inserting pass (paper, Section 3, Algorithm 1) and the lowering
// of its output to device launches (fused tile passes, data movement, plain
// gates).
//
// Reading of the pass (the paper leaves these points open):
//  * qubit q is local iff sigma(q) < m; a gate is local iff every qubit it acts
//    on non-diagonally is local (a control or CZ is diagonal), so a CNOT with a
//    global control and local target is local (Sections 2 and 4, Appendix C);
//  * DAG edges join every pair of gates that share a qubit and do not commute
//    exactly: gates commute when, on each shared qubit, both act diagonally or
//    both act as a matrix in span{I, X}, or when they are identical (Section 3);
//  * a candidate exchange (l, g) swaps the positions of qubits l and g; its
//    score is the number of remaining gates that become schedulable (local,
//    with every predecessor scheduled or itself counted);
//  * candidates run over l, then g, in ascending qubit index; the first strict
//    maximum wins; the fallback gate is the lowest-index ready gate.
//
// Only exchanges whose incoming qubit g is the non-diagonal target of a gate
// that is ready under the current placement (or becomes ready through gates
// already counted) can raise the score, so only those g are scored.  Other
// exchanges cannot beat the running maximum, and the chosen exchange is the
// one a full scan of all m(n-m) candidates picks.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <functional>
#include <queue>

#include "internal.h"

namespace qsim {

int matrix_action(const double *u)
{
    if (u[2] == 0 && u[3] == 0 && u[4] == 0 && u[5] == 0)
        return ACT_Z;
    if (u[0] == u[6] && u[1] == u[7] && u[2] == u[4] && u[3] == u[5])
        return ACT_X;
    return ACT_G;
}

GateInfo analyse(const qs_gate &g)
{
    GateInfo gi{};
    gi.kind = g.kind;
    gi.q0 = g.q0;
    gi.q1 = g.q1;
    gi.u = g.u;
    switch (g.kind) {
    case QS_GATE_U:
        gi.nq = 1;
        gi.act0 = matrix_action(g.u);
        gi.act1 = ACT_NONE;
        gi.target = gi.act0 == ACT_Z ? -1 : g.q0;
        break;
    case QS_GATE_CX:
        gi.nq = 2;
        gi.act0 = ACT_Z;
        gi.act1 = ACT_X;
        gi.target = g.q1;
        break;
    case QS_GATE_CZ:
        gi.nq = 2;
        gi.act0 = gi.act1 = ACT_Z;
        gi.target = -1;
        break;
    case QS_GATE_CU:
        gi.nq = 2;
        gi.act0 = ACT_Z;
        gi.act1 = matrix_action(g.u);
        gi.target = gi.act1 == ACT_Z ? -1 : g.q1;
        break;
    default:
        fail(QS_ERR_ARG, "unknown gate kind " + std::to_string(g.kind));
    }
    return gi;
}

static int act_on(const GateInfo &gi, int q)
{
    if (q == gi.q0)
        return gi.act0;
    if (gi.nq == 2 && q == gi.q1)
        return gi.act1;
    return ACT_NONE;
}

bool gates_commute(const qs_gate &a, const GateInfo &ia, const qs_gate &b, const GateInfo &ib)
{
    if (a.kind == b.kind && a.q0 == b.q0 && a.q1 == b.q1 && std::memcmp(a.u, b.u, sizeof a.u) == 0)
        return true;
    const int qa[2] = {ia.q0, ia.q1};
    for (int k = 0; k < ia.nq; ++k) {
        int tb = act_on(ib, qa[k]);
        if (tb == ACT_NONE)
            continue;
        int ta = k == 0 ? ia.act0 : ia.act1;
        if (!(ta == tb && (ta == ACT_Z || ta == ACT_X)))
            return false;
    }
    return true;
}

namespace {

Dag build_dag(const qs_gate *g, const std::vector<GateInfo> &gi, int n)
{
    const int ng = (int)gi.size();
    Dag d;
    d.pred.resize(ng);
    d.succ.resize(ng);
    std::vector<std::vector<int>> uses(n);
    // cut[q]: every gate on q before uses[q][cut[q]] is an ancestor of that
    // gate, so a gate that depends on it needs no edge from them (the edges
    // left out are implied, readiness is unchanged)
    std::vector<size_t> cut(n, 0);
    std::vector<int> seen(ng, -1);
    for (int v = 0; v < ng; ++v) {
        const int qs[2] = {gi[v].q0, gi[v].q1};
        bool all_pred[2] = {true, true};
        for (int k = 0; k < gi[v].nq; ++k) {
            const std::vector<int> &u = uses[qs[k]];
            // the cut gate commuting with v (an identical gate) implies nothing
            size_t lo = cut[qs[k]];
            if (lo < u.size() && gates_commute(g[u[lo]], gi[u[lo]], g[v], gi[v]))
                lo = 0;
            for (size_t i = lo; i < u.size(); ++i) {
                const int h = u[i];
                if (seen[h] == v) {
                    all_pred[k] = all_pred[k] && !d.pred[v].empty() &&
                                  std::find(d.pred[v].begin(), d.pred[v].end(), h) != d.pred[v].end();
                    continue;
                }
                seen[h] = v;
                if (!gates_commute(g[h], gi[h], g[v], gi[v]))
                    d.pred[v].push_back(h);
                else
                    all_pred[k] = false;
            }
            all_pred[k] = all_pred[k] && lo == cut[qs[k]];
        }
        std::sort(d.pred[v].begin(), d.pred[v].end());
        for (int h : d.pred[v])
            d.succ[h].push_back(v);
        for (int k = 0; k < gi[v].nq; ++k) {
            const int q = qs[k];
            // v acts on q with a general matrix and depends on every gate on q
            // from the cut on: every earlier gate on q is now its ancestor
            if (act_on(gi[v], q) == ACT_G && all_pred[k])
                cut[q] = uses[q].size();
            uses[q].push_back(v);
        }
    }
    return d;
}

inline bool is_local(const GateInfo &gi, const int *sigma, int m)
{
    return gi.target < 0 || sigma[gi.target] < m;
}

using MinHeap = std::priority_queue<int, std::vector<int>, std::greater<int>>;

}  // namespace

class PassState {
public:
    PassState(const std::vector<GateInfo> &gi, const Dag &d, int n, int m)
        : gi_(gi), d_(d), n_(n), m_(m), npend_(gi.size()), tmp_(gi.size(), -1), done_(gi.size(), 0)
    {
        for (size_t v = 0; v < gi.size(); ++v) {
            npend_[v] = (int)d.pred[v].size();
            if (npend_[v] == 0)
                frontier_.push_back((int)v);
        }
        remaining_ = (int64_t)gi.size();
    }

    int64_t remaining() const { return remaining_; }

    // Schedule every local gate whose predecessors are scheduled, in program
    // order (one sweep in index order reaches the fixed point).
    void sweep(const int *sigma, std::vector<int> &emitted)
    {
        MinHeap h(std::greater<int>(), frontier_);
        std::vector<int> blocked;
        while (!h.empty()) {
            int v = h.top();
            h.pop();
            if (is_local(gi_[v], sigma, m_)) {
                emitted.push_back(v);
                mark_done(v, &h);
            } else {
                blocked.push_back(v);
            }
        }
        frontier_.swap(blocked);
    }

    // Number of not-scheduled gates that become schedulable under sigma;
    // optionally collects the non-diagonal targets (qubits) of gates that are
    // reached (all predecessors done or counted) but are not local, and the
    // counted gates by cost class (gate_class).
    // The closure does not depend on the order gates are visited in, so a
    // plain work list replaces the program-order heap of sweep().
    int64_t closure(const int *sigma, std::vector<char> *reach_targets, int64_t *classes = nullptr)
    {
        work_.assign(frontier_.begin(), frontier_.end());
        touched_.clear();
        int64_t cnt = 0;
        while (!work_.empty()) {
            const int v = work_.back();
            work_.pop_back();
            if (!is_local(gi_[v], sigma, m_)) {
                if (reach_targets)
                    (*reach_targets)[gi_[v].target] = 1;
                continue;
            }
            ++cnt;
            if (classes)
                ++classes[gate_class(gi_[v])];
            for (int s : d_.succ[v]) {
                if (tmp_[s] < 0) {
                    tmp_[s] = npend_[s];
                    touched_.push_back(s);
                }
                if (--tmp_[s] == 0)
                    work_.push_back(s);
            }
        }
        for (int s : touched_)
            tmp_[s] = -1;
        return cnt;
    }

    // qs_pass_costs::in_pass class: 0 non-diagonal one-qubit, 1 two-qubit
    // with a non-diagonal target, 2 diagonal
    static int gate_class(const GateInfo &gi) { return gi.target < 0 ? 2 : gi.nq == 1 ? 0 : 1; }

    // lowest-index ready gate (Algorithm 1 fallback), not scheduled
    int first_ready() const { return *std::min_element(frontier_.begin(), frontier_.end()); }

    // lowest-index ready gate (Algorithm 1 fallback); schedules it
    int take_first_ready()
    {
        auto it = std::min_element(frontier_.begin(), frontier_.end());
        int v = *it;
        frontier_.erase(it);
        std::vector<int> newly;
        mark_done(v, nullptr, &newly);
        frontier_.insert(frontier_.end(), newly.begin(), newly.end());
        return v;
    }

private:
    void mark_done(int v, MinHeap *h, std::vector<int> *newly = nullptr)
    {
        done_[v] = 1;
        --remaining_;
        for (int s : d_.succ[v])
            if (--npend_[s] == 0) {
                if (h)
                    h->push(s);
                if (newly)
                    newly->push_back(s);
            }
    }

    const std::vector<GateInfo> &gi_;
    const Dag &d_;
    int n_, m_;
    std::vector<int> npend_, tmp_, touched_, work_;
    std::vector<char> done_;
    std::vector<int> frontier_;
    int64_t remaining_;
};


// One iteration at a time: apply every ready local gate, then insert one
// PermuteQubits (or, when no exchange helps, run one gate as global).
PassRunner::PassRunner(const qs_gate *g, int64_t ng, int n, int m, int r, int pinned, const std::vector<int> &sigma0,
                       const qs_pass_costs *costs)
    : n_(n), m_(m), r_(r), pinned_(pinned), gi_(ng), sigma_(sigma0)
{
    if (costs) {
        costed_ = true;
        costs_ = *costs;
    }
    for (int64_t v = 0; v < ng; ++v)
        gi_[v] = analyse(g[v]);
    dag_ = build_dag(g, gi_, n);
    ps_ = new PassState(gi_, dag_, n, m);
}

PassRunner::~PassRunner() { delete ps_; }

bool PassRunner::step(std::vector<Instr> &out)
{
    PassState &ps = *ps_;
    if (!swept_) {
        if (ps.remaining() == 0)
            return false;
        emitted_.clear();
        ps.sweep(sigma_.data(), emitted_);
        for (int v : emitted_)
            out.push_back(Instr{0, v, {}});
        stats_.n_apply += (int64_t)emitted_.size();
        swept_ = true;
        return ps.remaining() != 0;
    }
    swept_ = false;
    const int n = n_, m = m_;

    // the chain of Algorithm 1's exchanges (each strictly raising the count),
    // with the placement and count after each link
    std::vector<int> cur = sigma_, cand(n), best(n);
    std::vector<char> targets(n);
    std::vector<std::vector<int>> prefix;
    std::vector<int64_t> counts;
    int64_t base = 0;
    for (int step = 0; step < r_; ++step) {
        std::fill(targets.begin(), targets.end(), 0);
        ps.closure(cur.data(), &targets);
        int64_t best_a = base;
        bool found = false;
        for (int l = 0; l < n; ++l) {
            if (!(cur[l] < m && cur[l] >= pinned_))
                continue;
            for (int gq = 0; gq < n; ++gq) {
                if (cur[gq] < m || !targets[gq])
                    continue;
                cand = cur;
                cand[l] = cur[gq];
                cand[gq] = cur[l];
                int64_t a = ps.closure(cand.data(), nullptr);
                if (a > best_a) {
                    best_a = a;
                    best = cand;
                    found = true;
                }
            }
        }
        if (!found)
            break;
        cur = best;
        base = best_a;
        prefix.push_back(cur);
        counts.push_back(best_a);
    }
    // Algorithm 1 takes the whole chain, or the fallback gate when it is empty
    int take = (int)prefix.size();
    if (costed_ && !prefix.empty()) {
        // predicted time per gate of each prefix: the permutation's data
        // movement, the tile pass and its gates; against the first ready gate
        // as a launch of its own.  Ties keep the longer chain, then the chain.
        double best_rate = 0.0;
        for (int b = (int)prefix.size(); b >= 1; --b) {
            int64_t cls[3] = {0, 0, 0};
            const int64_t a = ps.closure(prefix[b - 1].data(), nullptr, cls);
            int changed = 0;
            for (int q = 0; q < n; ++q)
                changed += prefix[b - 1][q] != sigma_[q];
            const double t = costs_.move * (1.0 - std::ldexp(1.0, -(changed / 2))) + costs_.tile_pass +
                             cls[0] * costs_.in_pass[0] + cls[1] * costs_.in_pass[1] + cls[2] * costs_.in_pass[2];
            const double rate = t / (double)std::max<int64_t>(a, 1);
            if (b == (int)prefix.size() || rate < best_rate) {
                best_rate = rate;
                take = b;
            }
        }
        const int v = ps.first_ready();
        const int kind = gi_[v].kind;
        const double plain = costs_.plain[kind >= 0 && kind < 4 ? kind : 0];
        if (plain < best_rate)
            take = 0;
    }
    if (take > 0) {
        sigma_ = prefix[take - 1];
        out.push_back(Instr{1, -1, sigma_});
        ++stats_.n_perm;
        stats_.n_swaps += take;
    } else {
        int v = ps.take_first_ready();
        out.push_back(Instr{2, v, {}});
        ++stats_.n_global;
    }
    return true;
}

std::vector<Instr> run_pass(const qs_gate *g, int64_t ng, int n, int m, int r, int pinned,
                            const std::vector<int> &sigma0, PassStats *st)
{
    PassRunner pr(g, ng, n, m, r, pinned, sigma0);
    std::vector<Instr> out;
    while (pr.step(out)) {
    }
    if (st)
        *st = pr.stats();
    return out;
}

// ---------------------------------------------------------------------------
// lowering

int pass_reg_bits(int k, qs_dtype dt)
{
    // measured on MI355X (30 qubits, random layers): 16 complex128 amplitudes
    // per thread from 2^11-amplitude tiles up, fewer registers below; 16
    // complex64 amplitudes per thread
    if (dt == QS_C128)
        return k >= 11 ? 4 : 3;
    return 4;
}

void tile_shape(int k, qs_dtype dt, int reg_bits_opt, int *log_r, int *log_nt)
{
    int lr = reg_bits_opt > 0 ? reg_bits_opt : pass_reg_bits(k, dt);
    lr = std::min(lr, 5);
    lr = std::max(lr, k - 10);   // at most 1024 threads
    lr = std::min(lr, k - 6);    // at least one wavefront
    lr = std::max(lr, 1);
    *log_r = lr;
    *log_nt = k - lr;
}

namespace {

// A gate lowered to tile-local form, before register slots are assigned.
struct LGate {
    int kind;        // OP_U / OP_X / OP_DIAG / OP_NEG
    int tb;          // tile bit of the non-diagonal target (OP_U/OP_X), DIAG target tile bit or -1
    uint32_t cmask;
    uint64_t hmask, hbit;
    double m[8];
    int q[2], nq;    // logical qubits (for in-segment dependencies)
    int qtb[2];      // tile bit of each logical qubit, -1 outside the tile
    int src;         // index into the source gate array
};

LGate lower_gate(const qs_gate &g, const GateInfo &gi, const std::vector<int> &sigma_phys,
                 const std::vector<int> &tile_bit_of_pos)
{
    LGate L{};
    L.src = -1;
    L.nq = gi.nq;
    L.q[0] = gi.q0;
    L.q[1] = gi.q1;
    for (int k = 0; k < gi.nq; ++k)
        L.qtb[k] = tile_bit_of_pos[sigma_phys[L.q[k]]];
    std::memcpy(L.m, g.u, sizeof L.m);
    auto add_ctrl = [&](int q) {
        int p = sigma_phys[q];
        int tb = tile_bit_of_pos[p];
        if (tb >= 0)
            L.cmask |= 1u << tb;
        else
            L.hmask |= 1ull << p;
    };
    auto set_diag_target = [&](int q, const double *d0, const double *d1) {
        int p = sigma_phys[q];
        int tb = tile_bit_of_pos[p];
        L.kind = OP_DIAG;
        L.tb = tb;
        L.hbit = tb >= 0 ? 0 : (1ull << p);
        L.m[0] = d0[0];
        L.m[1] = d0[1];
        L.m[2] = d1[0];
        L.m[3] = d1[1];
    };
    auto need_tile = [&](int q) {
        int tb = tile_bit_of_pos[sigma_phys[q]];
        if (tb < 0)
            fail(QS_ERR_STATE, "internal: non-local target in tile segment");
        return tb;
    };
    switch (g.kind) {
    case QS_GATE_U:
        if (gi.act0 == ACT_Z) {
            set_diag_target(g.q0, &g.u[0], &g.u[6]);
        } else {
            L.kind = OP_U;
            L.tb = need_tile(g.q0);
        }
        break;
    case QS_GATE_CX:
        L.kind = OP_X;
        L.tb = need_tile(g.q1);
        add_ctrl(g.q0);
        break;
    case QS_GATE_CZ:
        L.kind = OP_NEG;
        L.tb = -1;
        add_ctrl(g.q0);
        add_ctrl(g.q1);
        break;
    case QS_GATE_CU:
        if (gi.act1 == ACT_Z) {
            set_diag_target(g.q1, &g.u[0], &g.u[6]);
        } else {
            L.kind = OP_U;
            L.tb = need_tile(g.q1);
        }
        add_ctrl(g.q0);
        break;
    }
    return L;
}

// ---------------------------------------------------------------------------
// Pending one-qubit factors (lowering only; the pass is unchanged).
//
// Every invertible 2x2 matrix M with M00 != 0 factors as
//   M = M00 diag(1, z) L(q) U(p),  U(p) = [[1, p], [0, 1]], L(q) = [[1, 0], [q, 1]],
// with p = M01 / M00, q = M10 M00 / det M and z = det M / M00^2 (multiply
// out: the product is [[M00, M01], [M10, M11]]).  The two shears update an
// amplitude pair (x, y) in place, x += p y and then y += q x, with 8 real
// multiply-adds instead of the 16 of a general complex 2x2, and need no
// temporary.  When |M01| > |M00| the same is done for M X = [[M01, M00],
// [M11, M10]] (det M X = -det M) and an exchange X on the qubit runs first
// (flagged on the op: an uncontrolled exchange on a register slot is a
// relabelling of slots and moves no data).  Pivoting on the larger entry of
// the first row keeps |p| <= 1.
//
// M also factors as M = (a I + b X) L(q) U(p) (or with an exchange first):
// N = (a I + b X)^-1 M must have N00 = 1 and det N = 1, which fixes a and b
// up to the two roots of a quadratic (solved below).  The left factor
// commutes with every operation that acts on the qubit as a matrix in
// span{I, X} (the target of a CNOT), where diag(1, z) does not.
//
// The lowering applies the shears of each uncontrolled one-qubit gate in a
// tile pass and keeps the left factor pending on the gate's qubit: diag(1, z)
// (with M00 moved into one scalar for the whole state) when the operations on
// the qubit up to its next one-qubit gate act on it diagonally (CZ, a
// control), a I + b X when they are all CNOT targets.  The stored state equals
// the true state with the pending factors and the scalar divided out.  The
// next one-qubit gate on the qubit absorbs its pending factor into its own
// matrix (host arithmetic, no device work).  An operation that does not
// commute with the pending factor needs it applied first: diag(1, z) before a
// non-diagonal target, as a multiplication of the amplitudes whose bit is 1
// (OP_PHASE), and a I + b X before a diagonal action or a general target, as a
// whole 2x2.  The latter cannot be needed before a diagonal action: such an
// operation between the gate and the next one-qubit gate on the qubit would
// have chosen the diagonal form, and any other is ordered before the gate or
// after that next gate by the commutation DAG (a diagonal action does not
// commute with a non-diagonal one-qubit gate).  The last one-qubit gate of each
// qubit is applied whole with its pending factor absorbed, and a gate applied
// whole also takes the scalar (it touches every amplitude), so the state is
// exact (up to rounding) when the program ends.  The stored amplitudes stay
// within a bounded factor of the true ones: a gate is applied whole instead
// when the new pending factor's condition number would exceed 4 for
// diag(1, z) (|z| outside [1/4, 4]) or 8 for a I + b X (|a + b| / |a - b| or its
// inverse; for unitary M the best root reaches 5.8), its determinant leave
// [1/16, 16], the scalar's magnitude [2^-8, 2^8], or |p|, |q| exceed 16,
// so that complex64 states keep at least 2^-(2n+8) of their magnitude range.
//
// a I + b X pending factors are used for complex128 states only, and for
// complex64 states with QS_OPT_X_FACTORS.  A diagonal
// pending factor scales each stored amplitude, so rounding errors stay
// relative to each amplitude; a I + b X mixes the two amplitudes of a pair,
// and with many qubits holding one at once the stored state is their tensor
// product's inverse applied to the true state: rounding errors come back
// amplified (measured on the 22-qubit layered workload: maximum amplitude
// error 2.6e-8 instead of 3.1e-9 in complex64, 1.5e-16 instead of 1.4e-17 in
// complex128).  Complex64 keeps the diagonal form and its accuracy; complex128
// stays near 1e-13 relative error.
struct PhaseFrame {
    using cd = std::complex<double>;
    static constexpr double Z_LO = 0.25, Z_HI = 4.0, S_LO = 1.0 / 256.0, S_HI = 256.0, Q_MAX = 16.0;
    static constexpr double DET_LO = 1.0 / 16.0, DET_HI = 16.0, K_X = 8.0, RESIDUAL = 1e-13;
    enum : int8_t { P_NONE = 0, P_DIAG = 1, P_XT = 2 };
    enum Action { A_DIAG, A_X, A_GEN };
    bool on = false;
    // pending factor per logical qubit: P_DIAG diag(1, z[q]); P_XT a[q] I + b[q] X
    std::vector<int8_t> type;
    std::vector<cd> z, a, b;
    std::vector<int64_t> u_left;   // non-diagonal one-qubit gates of q not yet lowered
    std::vector<char> prefer_x;    // per gate: its pending factor should commute with X
    cd scalar{1.0, 0.0};           // accumulated product of the pivots

    static bool absorbing(const qs_gate &g, const GateInfo &gi) { return g.kind == QS_GATE_U && gi.act0 != ACT_Z; }
    // how gate gi acts on qubit q (it acts on q)
    static Action action(const GateInfo &gi, int q)
    {
        const int act = q == gi.q0 ? gi.act0 : gi.act1;
        return act == ACT_Z ? A_DIAG : act == ACT_X && gi.nq == 2 ? A_X : A_GEN;
    }

    void init(const qs_gate *g, const std::vector<GateInfo> &gi, int64_t ng, int n, bool allow_x)
    {
        type.assign(n, P_NONE);
        z.assign(n, cd(1.0, 0.0));
        a.assign(n, cd(1.0, 0.0));
        b.assign(n, cd(0.0, 0.0));
        u_left.assign(n, 0);
        scalar = cd(1.0, 0.0);
        prefer_x.assign(ng, 0);
        // for each qubit, walking backwards: do the operations on it up to its
        // next one-qubit gate all act on it as CNOT targets (and is there one)?
        std::vector<int> state(n, 0);  // 0 none yet, 1 all X so far, 2 mixed
        for (int64_t v = ng - 1; v >= 0; --v) {
            const int qs[2] = {gi[v].q0, gi[v].q1};
            for (int k = 0; k < gi[v].nq; ++k) {
                const int q = qs[k];
                if (absorbing(g[v], gi[v])) {
                    prefer_x[v] = allow_x && state[q] == 1;
                    state[q] = 0;
                } else {
                    state[q] = action(gi[v], q) == A_X && state[q] != 2 ? 1 : 2;
                }
            }
            if (absorbing(g[v], gi[v]))
                ++u_left[g[v].q0];
        }
    }
    static cd at(const double *m, int i) { return cd(m[2 * i], m[2 * i + 1]); }
    static void put(double *m, int i, cd c)
    {
        m[2 * i] = c.real();
        m[2 * i + 1] = c.imag();
    }
    void clear(int q)
    {
        type[q] = P_NONE;
        z[q] = a[q] = cd(1.0, 0.0);
        b[q] = cd(0.0, 0.0);
    }
    // M = u P: the gate's matrix with qubit q's pending factor absorbed
    void absorb(int q, const double *u, cd M[4]) const
    {
        const cd u00 = at(u, 0), u01 = at(u, 1), u10 = at(u, 2), u11 = at(u, 3);
        if (type[q] == P_XT) {
            M[0] = u00 * a[q] + u01 * b[q];
            M[1] = u00 * b[q] + u01 * a[q];
            M[2] = u10 * a[q] + u11 * b[q];
            M[3] = u10 * b[q] + u11 * a[q];
        } else {
            M[0] = u00;
            M[1] = u01 * z[q];
            M[2] = u10;
            M[3] = u11 * z[q];
        }
    }
    // M = (a I + b X) L(q) U(p) X^x with the best-conditioned left factor;
    // false when none is within the bounds
    static bool factor_x(const cd M[4], cd *pa, cd *pb, cd *pp, cd *pq, bool *px)
    {
        double best = 0.0;
        bool found = false;
        for (int x = 0; x < 2; ++x) {
            // columns exchanged with the exchange first
            const cd m00 = x ? M[1] : M[0], m01 = x ? M[0] : M[1], m10 = x ? M[3] : M[2], m11 = x ? M[2] : M[3];
            const cd D = m00 * m11 - m01 * m10;
            // a m00 - b m10 = D and a^2 - b^2 = D:
            // b^2 (m10^2 - m00^2) + 2 D m10 b + D^2 - D m00^2 = 0
            const cd A = m10 * m10 - m00 * m00, B = 2.0 * D * m10, C = D * D - D * m00 * m00;
            if (std::abs(m00) == 0.0 || std::abs(D) == 0.0)
                continue;
            const cd disc = std::sqrt(B * B - 4.0 * A * C);
            for (int r = 0; r < 2; ++r) {
                const cd den = r ? -B + disc : -B - disc;  // b = 2C / den (stable for both roots)
                if (std::abs(den) == 0.0)
                    continue;
                const cd bb = 2.0 * C / den, aa = (D + bb * m10) / m00;
                const cd det = aa * aa - bb * bb;
                if (std::abs(det) == 0.0)
                    continue;
                // N = (a I - b X) M / det: N01 = p, N10 = q
                const cd p = (aa * m01 - bb * m11) / det, q = (aa * m10 - bb * m00) / det;
                const double e1 = std::abs(aa + bb), e2 = std::abs(aa - bb);
                if (e1 == 0.0 || e2 == 0.0)
                    continue;
                const double kappa = std::max(e1 / e2, e2 / e1), ad = std::abs(det);
                if (kappa > K_X || ad < DET_LO || ad > DET_HI || std::abs(p) > Q_MAX || std::abs(q) > Q_MAX)
                    continue;
                // the root can lose digits to cancellation: keep the candidate
                // only if (a I + b X) L(q) U(p) gives back the matrix
                const cd back[4] = {aa + bb * q, aa * p + bb * (1.0 + q * p), bb + aa * q, bb * p + aa * (1.0 + q * p)};
                const cd mm[4] = {m00, m01, m10, m11};
                double err = 0.0, scale = 0.0;
                for (int i = 0; i < 4; ++i) {
                    err = std::max(err, std::abs(back[i] - mm[i]));
                    scale = std::max(scale, std::abs(mm[i]));
                }
                if (err > RESIDUAL * scale)
                    continue;
                if (!found || kappa < best) {
                    found = true;
                    best = kappa;
                    *pa = aa;
                    *pb = bb;
                    *pp = p;
                    *pq = q;
                    *px = x != 0;
                }
            }
        }
        return found;
    }
    // Lower the uncontrolled one-qubit gate v (matrix u) on logical qubit q:
    // writes the op's kind and matrix fields (OP_SHEAR: m[0..1] = p, m[2..3] =
    // q; OP_U: the whole matrix) and *flip, true when an uncontrolled exchange
    // on q must run just before the op; updates the pending factor of q.
    // v < 0: the gate is applied whole.
    void one_qubit(int64_t v, int q, const double *u, int32_t *kind, double *m, bool *flip)
    {
        cd M[4];
        absorb(q, u, M);
        *flip = false;
        std::memset(m, 0, 8 * sizeof(double));
        if (--u_left[q] > 0 && v >= 0) {
            cd pa, pb, pp, pq;
            bool x;
            if (prefer_x[v] && factor_x(M, &pa, &pb, &pp, &pq, &x)) {
                *kind = OP_SHEAR;
                *flip = x;
                put(m, 0, pp);
                put(m, 1, pq);
                type[q] = P_XT;
                a[q] = pa;
                b[q] = pb;
                z[q] = cd(1.0, 0.0);
                return;
            }
            const cd det = M[0] * M[3] - M[1] * M[2];
            const bool xx = std::abs(M[1]) > std::abs(M[0]);
            const cd piv = xx ? M[1] : M[0];
            // with the exchange: M X = [[M01, M00], [M11, M10]], det M X = -det M
            const cd p = (xx ? M[0] : M[1]) / piv, qq = xx ? -M[3] * piv / det : M[2] * piv / det;
            const cd zn = xx ? -det / (piv * piv) : det / (piv * piv), sn = scalar * piv;
            const double az = std::abs(zn), as = std::abs(sn);
            if (std::abs(det) > 0.0 && az >= Z_LO && az <= Z_HI && as >= S_LO && as <= S_HI &&
                std::abs(qq) <= Q_MAX) {
                *kind = OP_SHEAR;
                *flip = xx;
                put(m, 0, p);
                put(m, 1, qq);
                type[q] = P_DIAG;
                z[q] = zn;
                a[q] = cd(1.0, 0.0);
                b[q] = cd(0.0, 0.0);
                scalar = sn;
                return;
            }
        }
        *kind = OP_U;
        for (int i = 0; i < 4; ++i)
            put(m, i, M[i] * scalar);
        scalar = cd(1.0, 0.0);
        clear(q);
    }
    // Before gate gi acts on q with the given action: what of q's pending
    // factor must be applied first, as a 2x2 matrix in out[8] (the record
    // layout of qs_gate.u).  Returns 0 (nothing), 1 (diag(1, z): a phase on
    // the amplitudes whose bit is 1, out[6..7] = z) or 2 (a whole 2x2).
    int settle(int q, Action act, double *out)
    {
        std::memset(out, 0, 8 * sizeof(double));
        if (type[q] == P_DIAG && act != A_DIAG) {
            put(out, 0, cd(1.0, 0.0));
            put(out, 3, z[q]);
            clear(q);
            return 1;
        }
        if (type[q] == P_XT && act != A_X) {
            put(out, 0, a[q]);
            put(out, 1, b[q]);
            put(out, 2, b[q]);
            put(out, 3, a[q]);
            clear(q);
            return 2;
        }
        return 0;
    }
};

// Order the gates of one tile pass and insert register re-layouts.  The gates
// may be reordered only along the commutation DAG restricted to the segment.
constexpr int LOOKAHEAD_TARGETS = 8;

// With lane_bits > 0, an uncontrolled one-qubit gate whose target sits on one
// of the lowest lane_bits thread-id bits of the current layout may run there
// through lane exchanges (OP_LANE, applied whole) instead of waiting for a
// re-layout: when every ready gate that needs a register slot is such a gate
// (so the re-layout is put off), or, with lane_eager, as soon as it is ready.
int schedule_segment(const std::vector<LGate> &lg, const qs_gate *g, const std::vector<GateInfo> &gi,
                     int k, int log_r, std::vector<TileOp> &ops, PhaseFrame &pf, int lane_bits, bool lane_eager)
{
    const int cnt = (int)lg.size();
    // in-segment predecessors
    std::vector<std::vector<int>> pred(cnt);
    for (int v = 0; v < cnt; ++v)
        for (int h = 0; h < v; ++h) {
            bool share = false;
            for (int a = 0; a < lg[h].nq; ++a)
                for (int b = 0; b < lg[v].nq; ++b)
                    share |= lg[h].q[a] == lg[v].q[b];
            if (share && !gates_commute(g[lg[h].src], gi[lg[h].src], g[lg[v].src], gi[lg[v].src]))
                pred[v].push_back(h);
        }
    std::vector<char> emitted(cnt, 0);
    int left = cnt, remaps = 0;
    const size_t seg_begin = ops.size();
    const int R = log_r;
    int regs[8];
    int thread_of[16];  // tile bit -> thread-id bit of the current layout (-1: a register slot)
    bool have = false;
    auto in_regs = [&](int tb) {
        if (!have)
            return -1;
        for (int s = 0; s < R; ++s)
            if (regs[s] == tb)
                return s;
        return -1;
    };
    auto ready = [&](int v) {
        for (int h : pred[v])
            if (!emitted[h])
                return false;
        return true;
    };
    auto needs_reg = [&](int v) { return lg[v].kind == OP_U || lg[v].kind == OP_X; };
    // thread-id bit of gate v's target when it may run as OP_LANE, else -1
    auto lane_of = [&](int v) {
        const LGate &L = lg[v];
        if (lane_bits <= 0 || !have || L.kind != OP_U || L.cmask != 0 || L.hmask != 0 ||
            g[L.src].kind != QS_GATE_U || in_regs(L.tb) >= 0)
            return -1;
        const int i = thread_of[L.tb];
        return i >= 0 && i < lane_bits ? i : -1;
    };
    auto emit_lane = [&](int v, int i) {
        TileOp op{};
        op.kind = OP_LANE;
        op.tlane = (uint32_t)i;
        std::memcpy(op.m, lg[v].m, sizeof op.m);
        if (pf.on) {
            // applied whole: q's pending factor and the scalar are taken
            const qs_gate &src = g[lg[v].src];
            int32_t kind = 0;
            bool flip = false;
            pf.one_qubit(-1, src.q0, src.u, &kind, op.m, &flip);
        }
        ops.push_back(op);
        emitted[v] = 1;
        --left;
    };
    while (left > 0) {
        bool progress = true;
        while (progress) {
            progress = false;
            for (int v = 0; v < cnt; ++v) {
                if (emitted[v] || !ready(v))
                    continue;
                int slot = -1;
                if (!have)
                    continue;   // ops act on register data: a layout must exist
                if (lane_eager) {
                    const int i = lane_of(v);
                    if (i >= 0) {
                        emit_lane(v, i);
                        progress = true;
                        continue;
                    }
                }
                if (needs_reg(v)) {
                    slot = in_regs(lg[v].tb);
                    if (slot < 0)
                        continue;
                }
                TileOp op{};
                op.kind = lg[v].kind;
                // split the in-tile controls into register slots and thread bits
                for (int b = 0; b < k; ++b) {
                    if (!((lg[v].cmask >> b) & 1u))
                        continue;
                    const int s = in_regs(b);
                    if (s >= 0)
                        op.rmask |= 1u << s;
                    else
                        op.lmask |= 1u << b;
                }
                if (needs_reg(v)) {
                    op.slot = slot;
                } else if (lg[v].kind == OP_DIAG) {
                    const int tb = lg[v].tb;
                    const int s = tb >= 0 ? in_regs(tb) : -1;
                    op.slot = tb < 0 ? -2 : s >= 0 ? s : -1;
                    op.tlane = tb >= 0 && s < 0 ? 1u << tb : 0u;
                } else {
                    op.slot = 0;
                }
                op.hmask = lg[v].hmask;
                op.hbit = lg[v].hbit;
                std::memcpy(op.m, lg[v].m, sizeof op.m);
                if (pf.on) {
                    const int64_t sv = lg[v].src;
                    const qs_gate &src = g[sv];
                    if (PhaseFrame::absorbing(src, gi[sv])) {
                        bool flip = false;
                        pf.one_qubit(sv, src.q0, src.u, &op.kind, op.m, &flip);
                        op.tlane = flip ? 1u : 0u;
                    } else {
                        // pending factors that do not commute with this
                        // operation go first (on a register slot: the
                        // qubit is the operation's target, see PhaseFrame)
                        for (int a = 0; a < lg[v].nq; ++a) {
                            double sm[8];
                            const int q = lg[v].q[a];
                            const int how = pf.settle(q, PhaseFrame::action(gi[sv], q), sm);
                            if (how == 0)
                                continue;
                            const int s = lg[v].qtb[a] >= 0 ? in_regs(lg[v].qtb[a]) : -1;
                            if (s < 0)
                                fail(QS_ERR_STATE, "internal: pending factor on a qubit outside the register slots");
                            TileOp po{};
                            po.slot = s;
                            if (how == 1) {
                                po.kind = OP_PHASE;
                                po.m[0] = sm[6];
                                po.m[1] = sm[7];
                            } else {
                                po.kind = OP_U;
                                std::memcpy(po.m, sm, sizeof po.m);
                            }
                            ops.push_back(po);
                        }
                    }
                }
                // a shear right after a shear on another slot of this pass
                // shares its record (one fetch and dispatch for two gates)
                if (op.kind == OP_SHEAR && ops.size() > seg_begin && ops.back().kind == OP_SHEAR &&
                    ops.back().slot != op.slot) {
                    TileOp &prev = ops.back();
                    prev.kind = OP_SHEAR2;
                    prev.aux = (uint32_t)op.slot | (op.tlane ? 256u : 0u);
                    std::memcpy(prev.m + 4, op.m, 4 * sizeof(double));
                } else {
                    ops.push_back(op);
                }
                emitted[v] = 1;
                --left;
                progress = true;
            }
        }
        if (left == 0)
            break;
        if (lane_bits > 0 && have) {
            // every blocked ready gate can run on its lane bit: no re-layout yet
            std::vector<std::pair<int, int>> lane;
            bool all = true;
            for (int v = 0; v < cnt && all; ++v)
                if (!emitted[v] && ready(v) && needs_reg(v)) {
                    const int i = lane_of(v);
                    all = i >= 0;
                    lane.emplace_back(v, i);
                }
            if (all && !lane.empty()) {
                for (const auto &vi : lane)
                    emit_lane(vi.first, vi.second);
                continue;
            }
        }
        // re-layout: targets of ready gates first, then of later gates
        std::vector<int> want;
        auto add = [&](int tb) {
            if (tb >= 0 && std::find(want.begin(), want.end(), tb) == want.end())
                want.push_back(tb);
        };
        for (int v = 0; v < cnt; ++v)
            if (!emitted[v] && ready(v) && needs_reg(v))
                add(lg[v].tb);
        if ((int)want.size() > R) {
            // more ready targets than register slots: of the first LOOK of
            // them, keep the R that let the most gates run before the next
            // re-layout (ties: program order)
            const int LOOK = std::min((int)want.size(), LOOKAHEAD_TARGETS);
            std::vector<int> best_set(want.begin(), want.begin() + R);
            int best_run = -1;
            std::vector<char> em(cnt);
            for (uint32_t sel = 0; sel < (1u << LOOK); ++sel) {
                if (__builtin_popcount(sel) != R)
                    continue;
                std::vector<int> set;
                for (int b = 0; b < LOOK; ++b)
                    if ((sel >> b) & 1u)
                        set.push_back(want[b]);
                std::copy(emitted.begin(), emitted.end(), em.begin());
                int run = 0;
                for (bool more = true; more;) {
                    more = false;
                    for (int v = 0; v < cnt; ++v) {
                        if (em[v])
                            continue;
                        bool rd = true;
                        for (int h : pred[v])
                            rd &= em[h] != 0;
                        if (!rd)
                            continue;
                        if (needs_reg(v) && std::find(set.begin(), set.end(), lg[v].tb) == set.end())
                            continue;
                        em[v] = 1;
                        ++run;
                        more = true;
                    }
                }
                // subsets in increasing order of their lowest chosen index
                // come later for equal counts, so only a larger count wins
                if (run > best_run) {
                    best_run = run;
                    best_set = set;
                }
            }
            want = best_set;
        }
        for (int v = 0; v < cnt && (int)want.size() < R; ++v)
            if (!emitted[v] && needs_reg(v))
                add(lg[v].tb);
        if (have)
            for (int s = 0; s < R; ++s)
                add(regs[s]);
        for (int b = k - 1; b >= 0 && (int)want.size() < R; --b)
            add(b);
        TileOp op{};
        op.kind = OP_REMAP;
        uint32_t packed = 0;
        for (int s = 0; s < R; ++s) {
            regs[s] = want[s];
            packed |= (uint32_t)want[s] << (4 * s);
        }
        op.rmask = packed;
        uint32_t words[16] = {};
        for (int s = 0; s < R; ++s)
            words[s] = lds_swizzle(1u << want[s], k);
        std::memcpy(op.m, words, sizeof op.m);
        // thread-id bits take the other tile bits in ascending order
        uint64_t lanes = 0;
        for (int b = 0, i = 0; b < k; ++b) {
            bool reg = false;
            for (int s = 0; s < R; ++s)
                reg |= regs[s] == b;
            thread_of[b] = reg ? -1 : i;
            if (!reg)
                lanes |= (uint64_t)b << (4 * i++);
        }
        op.hbit = lanes;
        ops.push_back(op);
        have = true;
        ++remaps;
    }
    return remaps;
}

// Wavefront-local re-layouts.  The thread-id bits above the lane bits (6 and
// up) number the wavefronts of a workgroup.  A re-layout that leaves the same
// tile bits on them moves amplitudes only between the lanes and registers of
// each wavefront: every wavefront reads back from LDS only the slots it wrote
// itself, and a wavefront's LDS instructions run in order, so the re-layout
// needs no barrier (OP_REMAP with aux bit REMAP_WAVE_LOCAL).  The register
// sets of the segment's re-layouts are fixed by the scheduler; this picks the
// tile bits of the wavefront bits: at each re-layout that must move them
// (its register set takes one of them, or the first of the pass), the tile
// bits outside its register set and outside the lowest `low` bits (which stay
// on lane bits for whole 128-byte lines at load and store) whose next use in
// a register set comes last; the other thread bits take the remaining tile
// bits in ascending order.
// Lane order of the tile bits outside `taken`: the lowest `low` first (in
// ascending order), then, up to bank_bits lanes, the lowest bit whose LDS bank
// bits (the low bank_bits bits of lds_swizzle of the bit) are independent over
// GF(2) of those of the lanes already placed, so that the lanes one LDS access
// serves together (2^bank_bits of them: 128 bytes of elements) hit distinct
// banks wherever the free bits allow; the rest in ascending order.
std::vector<int> bank_lane_order(int k, uint32_t taken, int low, int bank_bits)
{
    std::vector<int> order;
    std::vector<char> used(k, 0);
    uint32_t basis[8] = {};  // XOR basis of the placed lanes' bank bits, by leading bit
    auto reduces_to_zero = [&](int b) {
        uint32_t v = lds_swizzle(1u << b, k) & ((1u << bank_bits) - 1u);
        for (int t = bank_bits - 1; t >= 0 && v; --t)
            if ((v >> t) & 1u)
                v = basis[t] ? v ^ basis[t] : v;
        return v == 0;
    };
    auto insert = [&](int b) {
        uint32_t v = lds_swizzle(1u << b, k) & ((1u << bank_bits) - 1u);
        for (int t = bank_bits - 1; t >= 0 && v; --t)
            if ((v >> t) & 1u) {
                if (!basis[t]) {
                    basis[t] = v;
                    break;
                }
                v ^= basis[t];
            }
        order.push_back(b);
        used[b] = 1;
    };
    for (int b = 0; b < low && b < k; ++b)
        if (!((taken >> b) & 1u))
            insert(b);
    while ((int)order.size() < bank_bits) {
        int pick = -1;
        for (int b = 0; b < k && pick < 0; ++b)
            if (!used[b] && !((taken >> b) & 1u) && !reduces_to_zero(b))
                pick = b;
        if (pick < 0)
            break;
        insert(pick);
    }
    for (int b = 0; b < k; ++b)
        if (!used[b] && !((taken >> b) & 1u))
            order.push_back(b);
    return order;
}

void assign_wave_bits(std::vector<TileOp> &ops, size_t begin, int k, int log_r, int log_nt, int low, int bank_bits)
{
    const int nw = log_nt - 6;
    if (nw <= 0)
        return;
    std::vector<size_t> rl;
    for (size_t i = begin; i < ops.size(); ++i)
        if (ops[i].kind == OP_REMAP)
            rl.push_back(i);
    std::vector<uint32_t> sets(rl.size(), 0u);
    for (size_t j = 0; j < rl.size(); ++j)
        for (int s = 0; s < log_r; ++s)
            sets[j] |= 1u << ((ops[rl[j]].rmask >> (4 * s)) & 15u);
    uint32_t W = 0;
    for (size_t j = 0; j < rl.size(); ++j) {
        TileOp &op = ops[rl[j]];
        const bool keep = j > 0 && W != 0 && (sets[j] & W) == 0;
        if (!keep) {
            // candidates by next use (never: past the end); on ties bits with no
            // LDS bank bits first (they cannot spread a lane access over banks),
            // then higher bits
            std::vector<std::pair<size_t, int>> cand;
            for (int b = k - 1; b >= low; --b) {
                if ((sets[j] >> b) & 1u)
                    continue;
                size_t next = rl.size();
                for (size_t t = j + 1; t < rl.size(); ++t)
                    if ((sets[t] >> b) & 1u) {
                        next = t;
                        break;
                    }
                cand.emplace_back(next, b);
            }
            if ((int)cand.size() < nw) {
                W = 0;  // keep the ascending map
                continue;
            }
            auto no_bank = [&](int b) { return (lds_swizzle(1u << b, k) & ((1u << bank_bits) - 1u)) == 0; };
            std::stable_sort(cand.begin(), cand.end(),
                             [&](const std::pair<size_t, int> &a, const std::pair<size_t, int> &b) {
                                 if (a.first != b.first)
                                     return a.first > b.first;
                                 return no_bank(a.second) && !no_bank(b.second);
                             });
            W = 0;
            for (int i = 0; i < nw; ++i)
                W |= 1u << cand[i].second;
        }
        // lanes: the lowest `low` tile bits first, then bits that give the
        // lanes one LDS access serves together distinct banks, then the rest
        std::vector<int> order = bank_lane_order(k, sets[j] | W, low, bank_bits);
        for (int b = 0; b < k; ++b)
            if ((W >> b) & 1u)
                order.push_back(b);
        uint64_t lanes = 0;
        for (size_t i = 0; i < order.size(); ++i)
            lanes |= (uint64_t)order[i] << (4 * i);
        op.hbit = lanes;
        op.aux = keep ? REMAP_WAVE_LOCAL : 0u;
    }
}

// Tile bits that must be thread bits for each load or store instruction to
// move runs of DIRECT_RUN_BYTES contiguous bytes, and whether the tile's
// lowest positions are the lowest physical positions (else no run is that
// long whatever the layout).
int direct_low_bits(qs_dtype dt)
{
    const int esize = dt == QS_C64 ? 8 : 16;
    int low = 0;
    while ((esize << low) < DIRECT_RUN_BYTES)
        ++low;
    return low;
}
bool low_positions_contiguous(const Launch &L, int low)
{
    bool contiguous = true;
    for (int b = 0; b < low && b < L.k; ++b)
        contiguous &= L.pos[b] == b;
    return contiguous;
}

// The layout in force after the launch's last operation: register tile bits
// per slot and tile bit per thread bit (the last OP_REMAP and the OP_LSWAPs
// after it); false when the launch has no OP_REMAP.
bool final_layout(const Launch &L, const std::vector<TileOp> &ops, int *regs, int *lanes)
{
    const TileOp *o = ops.data() + L.op_begin;
    int last = -1;
    for (int i = L.op_count - 1; i >= 0 && last < 0; --i)
        if (o[i].kind == OP_REMAP)
            last = i;
    if (last < 0)
        return false;
    for (int s = 0; s < L.log_r; ++s)
        regs[s] = (int)((o[last].rmask >> (4 * s)) & 15u);
    for (int i = 0; i < L.log_nt; ++i)
        lanes[i] = (int)((o[last].hbit >> (4 * i)) & 15u);
    for (int i = last + 1; i < L.op_count; ++i)
        if (o[i].kind == OP_LSWAP)
            std::swap(regs[o[i].slot], lanes[o[i].tlane]);
    return true;
}

// When the last layout of a tile pass keeps one or two of the lowest tile
// bits in register slots, the store would go through an LDS re-layout to the
// plain layout.  Exchanging those slot bits with lane bits 4 and 5 of the
// wavefront (OP_LSWAP: cross-lane swaps in registers, no LDS and no barrier)
// puts them on thread bits instead, so the tile is stored straight from
// registers: the eight (complex128) or sixteen (complex64) amplitudes of a
// 128-byte line then sit in lanes of one store instruction.
void append_store_lane_swaps(Launch &L, std::vector<TileOp> &ops, qs_dtype dt)
{
    const int low = direct_low_bits(dt);
    if (L.op_count == 0 || !low_positions_contiguous(L, low) || L.log_nt < 6)
        return;
    int regs[8], lanes[16];
    if (!final_layout(L, ops, regs, lanes))
        return;
    std::vector<int> slots;
    for (int s = 0; s < L.log_r; ++s)
        if (regs[s] < low)
            slots.push_back(s);
    std::vector<int> free_lanes;
    for (int b : {5, 4})
        if (lanes[b] >= low)
            free_lanes.push_back(b);
    if (slots.empty() || slots.size() > free_lanes.size())
        return;
    for (size_t i = 0; i < slots.size(); ++i) {
        const int s = slots[i], b = free_lanes[i];
        TileOp op{};
        op.kind = OP_LSWAP;
        op.slot = s;
        op.tlane = (uint32_t)b;
        op.lmask = 1u << lanes[b];
        op.rmask = 1u << regs[s];
        const uint32_t w = lds_swizzle(1u << lanes[b], L.k);
        std::memcpy(op.m, &w, sizeof w);
        ops.push_back(op);
        ++L.op_count;
        std::swap(regs[s], lanes[b]);
    }
}

// A tile is loaded straight into the layout of its first OP_REMAP (and stored
// straight from its final layout) when the thread bits of that layout include
// the lowest tile bits, so that each load or store instruction still moves
// runs of DIRECT_RUN_BYTES contiguous bytes.  Otherwise it is loaded (stored)
// in tile-local index order j * NT + tid and goes through LDS.
void set_direct_io(Launch &L, const std::vector<TileOp> &ops, qs_dtype dt)
{
    const int low = direct_low_bits(dt);
    const bool contiguous = low_positions_contiguous(L, low);
    auto covers_low = [&](const int *regs) {
        for (int s = 0; s < L.log_r; ++s)
            if (regs[s] < low)
                return false;
        return contiguous;
    };
    // positions of a layout given by register tile bits and lane tile bits
    auto layout = [&](const int *regs, const int *lanes, uint8_t *lane, uint8_t *reg) {
        for (int i = 0; i < L.log_nt; ++i)
            lane[i] = (uint8_t)L.pos[lanes[i]];
        for (int s = 0; s < L.log_r; ++s)
            reg[s] = (uint8_t)L.pos[regs[s]];
    };
    auto plain = [&](uint8_t *lane, uint8_t *reg) {
        for (int i = 0; i < L.log_nt; ++i)
            lane[i] = (uint8_t)L.pos[i];
        for (int s = 0; s < L.log_r; ++s)
            reg[s] = (uint8_t)L.pos[L.log_nt + s];
    };
    L.io = contiguous ? 8u : 0u;
    plain(L.ld_lane, L.ld_reg);
    plain(L.st_lane, L.st_reg);
    const TileOp *o = ops.data() + L.op_begin;
    if (L.op_count == 0 || o[0].kind != OP_REMAP)
        return;
    int regs[8], lanes[16];
    for (int s = 0; s < L.log_r; ++s)
        regs[s] = (int)((o[0].rmask >> (4 * s)) & 15u);
    for (int i = 0; i < L.log_nt; ++i)
        lanes[i] = (int)((o[0].hbit >> (4 * i)) & 15u);
    if (covers_low(regs)) {
        L.io |= 1u;
        layout(regs, lanes, L.ld_lane, L.ld_reg);
    }
    if (final_layout(L, ops, regs, lanes) && covers_low(regs)) {
        L.io |= 2u;
        layout(regs, lanes, L.st_lane, L.st_reg);
    }
}

}  // namespace

void tile_args_from_launch(const Launch &L, TileArgs &a)
{
    a.n_ops = L.op_count;
    for (int b = 0; b < 16; ++b)
        a.pos[b] = (uint8_t)(b < L.k ? L.pos[b] : 0);
    a.io = L.io;
    for (int i = 0; i < 16; ++i) {
        a.ld_lane[i] = L.ld_lane[i];
        a.st_lane[i] = L.st_lane[i];
    }
    for (int s = 0; s < 8; ++s) {
        a.ld_reg[s] = L.ld_reg[s];
        a.st_reg[s] = L.st_reg[s];
    }
}

void tile_args_for_positions(const std::vector<int> &pos, int log_nt, int log_r, TileArgs &a)
{
    Launch L;
    L.type = L_TILE;
    L.k = (int)pos.size();
    L.log_nt = log_nt;
    L.log_r = log_r;
    L.pos = pos;
    set_direct_io(L, {}, QS_C128);
    tile_args_from_launch(L, a);
}

void tile_args_identity(int k, int log_nt, int log_r, TileArgs &a)
{
    std::vector<int> pos(k);
    for (int b = 0; b < k; ++b)
        pos[b] = b;
    tile_args_for_positions(pos, log_nt, log_r, a);
}

void compile_program(const qs_gate *g, int64_t ng, int n, qs_dtype dt, const int *sigma0_in,
                     const qs_run_opts &o, Program &p, const std::function<void(Program &)> &progress,
                     const qs_pass_costs *costs)
{
    auto t0 = std::chrono::steady_clock::now();
    if (n < 1 || n > MAX_COMPILE_QUBITS)
        fail(QS_ERR_ARG, "n out of range");
    p.n = n;
    p.dt = dt;
    if (o.flags & ~(QS_OPT_FULL_MATRICES | QS_OPT_LANE_GATES | QS_OPT_LANE_GATES_WIDE | QS_OPT_LANE_EAGER |
                    QS_OPT_FROM_ZERO | QS_OPT_X_FACTORS))
        fail(QS_ERR_ARG, "unknown flags");
    p.opts = o;
    p.sigma0.resize(n);
    for (int q = 0; q < n; ++q)
        p.sigma0[q] = sigma0_in ? sigma0_in[q] : q;
    {
        std::vector<char> seen(n, 0);
        for (int q = 0; q < n; ++q) {
            if (p.sigma0[q] < 0 || p.sigma0[q] >= n || seen[p.sigma0[q]])
                fail(QS_ERR_ARG, "sigma0 is not a permutation");
            seen[p.sigma0[q]] = 1;
        }
    }
    std::vector<GateInfo> gi(ng);
    for (int64_t v = 0; v < ng; ++v) {
        const qs_gate &x = g[v];
        if (x.q0 < 0 || x.q0 >= n)
            fail(QS_ERR_ARG, "gate " + std::to_string(v) + ": qubit out of range");
        if (x.kind != QS_GATE_U && (x.q1 < 0 || x.q1 >= n || x.q1 == x.q0))
            fail(QS_ERR_ARG, "gate " + std::to_string(v) + ": bad second qubit");
        gi[v] = analyse(x);
    }
    p.stats = qs_program_stats{};
    p.stats.n_gates = ng;
    p.launches.clear();
    p.ops.clear();
    std::vector<int> sphys = p.sigma0;

    PhaseFrame pf;
    auto plain = [&](int64_t v) {
        Launch L;
        L.type = L_PLAIN;
        L.gate = g[v];
        L.gate.q0 = sphys[g[v].q0];
        L.gate.q1 = g[v].kind == QS_GATE_U ? -1 : sphys[g[v].q1];
        if (pf.on) {
            if (PhaseFrame::absorbing(g[v], gi[v])) {
                // one launch of the whole matrix with the pending factor absorbed
                int32_t kind = OP_U;
                bool flip = false;
                pf.one_qubit(-1, g[v].q0, g[v].u, &kind, L.gate.u, &flip);
            } else {
                // pending factors that do not commute with the gate go first,
                // each as a one-qubit launch of its own
                const int qs[2] = {g[v].q0, g[v].q1};
                for (int a = 0; a < gi[v].nq; ++a) {
                    Launch D;
                    D.type = L_PLAIN;
                    D.gate = qs_gate{};
                    if (pf.settle(qs[a], PhaseFrame::action(gi[v], qs[a]), D.gate.u) == 0)
                        continue;
                    D.gate.kind = QS_GATE_U;
                    D.gate.q0 = sphys[qs[a]];
                    D.gate.q1 = -1;
                    p.launches.push_back(D);
                    ++p.stats.n_plain;
                }
            }
        }
        p.launches.push_back(L);
        ++p.stats.n_plain;
    };

    if (o.form == QS_FORM_PLAIN) {
        for (int64_t v = 0; v < ng; ++v) {
            p.instrs.push_back(Instr{0, (int)v, {}});
            plain(v);
        }
        p.sigma_final = sphys;
        p.stats.n_apply = ng;
    } else if (o.form == QS_FORM_PASS) {
        const int k = std::min(o.k_tile, n);
        if (k < 1)
            fail(QS_ERR_ARG, "k_tile must be >= 1");
        if (o.max_swaps < 0)
            fail(QS_ERR_ARG, "max_swaps must be >= 0");
        if (o.pinned < 0 || o.pinned > k)
            fail(QS_ERR_ARG, "pinned must be in [0, k_tile]");
        if (o.perm_exec != QS_PERM_MOVE && o.perm_exec != QS_PERM_RELABEL)
            fail(QS_ERR_ARG, "unknown perm_exec");

        // tile passes need 7 <= k and a tile that fits in one CU's LDS; a larger
        // local set (e.g. a pass planned for several devices) runs its
        // segments gate by gate
        const bool tiled = k >= MIN_TILE_BITS && (size_t(dt == QS_C64 ? 8 : 16) << k) <= MAX_TILE_BYTES;
        int log_r = 0, log_nt = 0;
        if (tiled)
            tile_shape(k, dt, o.reg_bits, &log_r, &log_nt);
        std::vector<int> spass = p.sigma0;
        size_t i = 0;
        // reduced one-qubit updates only where tile passes run them
        pf.on = tiled && (o.flags & QS_OPT_FULL_MATRICES) == 0;
        if (pf.on)
            pf.init(g, gi, ng, n, dt == QS_C128 || (o.flags & QS_OPT_X_FACTORS) != 0);
        const int lane_bits = (o.flags & QS_OPT_LANE_GATES_WIDE) ? 4 : (o.flags & QS_OPT_LANE_GATES) ? 2 : 0;
        const bool lane_eager = (o.flags & QS_OPT_LANE_EAGER) != 0;
        // Lower the instructions from i on.  A run of ApplyGate instructions is
        // a complete segment once an instruction of another kind follows it
        // (or, with final, at the end).
        auto lower = [&](bool final) {
            while (i < p.instrs.size()) {
                const Instr &I = p.instrs[i];
                if (I.type == 1) {
                    spass = I.sigma;
                    if (o.perm_exec == QS_PERM_MOVE) {
                        Launch L;
                        L.type = L_MOVE;
                        L.pi.resize(n);
                        for (int q = 0; q < n; ++q)
                            L.pi[sphys[q]] = spass[q];
                        p.launches.push_back(L);
                        ++p.stats.n_move_passes;
                        sphys = spass;
                    }
                    ++i;
                    continue;
                }
                if (I.type == 2) {
                    plain(I.gate);
                    ++i;
                    continue;
                }
                // a run of local ApplyGate instructions = one segment
                size_t j = i;
                while (j < p.instrs.size() && p.instrs[j].type == 0)
                    ++j;
                if (j == p.instrs.size() && !final)
                    return;
                if (!tiled) {
                    for (size_t t = i; t < j; ++t)
                        plain(p.instrs[t].gate);
                    i = j;
                    continue;
                }
                // tile positions: physical positions of the k local qubits
                std::vector<int> pos;
                for (int q = 0; q < n; ++q)
                    if (spass[q] < k)
                        pos.push_back(sphys[q]);
                std::sort(pos.begin(), pos.end());
                std::vector<int> tbit(n, -1);
                for (int b = 0; b < k; ++b)
                    tbit[pos[b]] = b;
                const size_t chunk = o.max_fuse > 0 ? (size_t)o.max_fuse : (j - i);
                for (size_t c0 = i; c0 < j; c0 += chunk) {
                    size_t c1 = std::min(j, c0 + chunk);
                    std::vector<LGate> lg;
                    for (size_t t = c0; t < c1; ++t) {
                        int v = p.instrs[t].gate;
                        LGate L = lower_gate(g[v], gi[v], sphys, tbit);
                        L.src = v;
                        lg.push_back(L);
                    }
                    Launch L;
                    L.type = L_TILE;
                    L.k = k;
                    L.log_r = log_r;
                    L.log_nt = log_nt;
                    L.pos = pos;
                    L.op_begin = (int)p.ops.size();
                    p.stats.n_remaps += schedule_segment(lg, g, gi, k, log_r, p.ops, pf, lane_bits, lane_eager);
                    // lane gates name thread bits of the ascending map
                    if (lane_bits == 0)
                        assign_wave_bits(p.ops, (size_t)L.op_begin, k, log_r, log_nt, direct_low_bits(dt),
                                         dt == QS_C64 ? 5 : 4);
                    L.op_count = (int)p.ops.size() - L.op_begin;
                    append_store_lane_swaps(L, p.ops, dt);
                    set_direct_io(L, p.ops, dt);
                    p.launches.push_back(L);
                    ++p.stats.n_tile_passes;
                }
                i = j;
            }
        };
        // the pass and the lowering advance together, so a caller can start
        // the first launches while later permutations are still being chosen
        PassRunner pr(g, ng, n, k, o.max_swaps, o.pinned, p.sigma0, costs);
        bool more = true;
        while (more) {
            more = pr.step(p.instrs);
            // a closed run of ApplyGate instructions is lowered (and may be
            // launched) before the PermuteQubits after it is chosen
            lower(!more || pr.run_closed());
            if (progress)
                progress(p);
        }
        const PassStats &ps = pr.stats();
        p.stats.n_apply = ps.n_apply;
        p.stats.n_perm = ps.n_perm;
        p.stats.n_global = ps.n_global;
        p.stats.n_swaps = ps.n_swaps;
        p.sigma_final = sphys;
    } else {
        fail(QS_ERR_ARG, "unknown form");
    }
    auto t1 = std::chrono::steady_clock::now();
    p.stats.compile_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
}

}  // namespace qsim
