// Batched gradients of independent problems of uneven size (grid, shots,
// receivers, time steps): the gradient evaluation of Secs. 2.1 and 3.3 for
// many models at once.
//
// A plan records, for every problem, the same sequence the single-problem
// gradient issues (coefficients, forward sweep with checkpoints, residual
// and misfit, adjoint sweep with segment re-forward, gradient scaling), each
// operation tagged with its position in a common schedule: all problems
// share one checkpoint interval, so their stencil passes line up pass by
// pass.  Passes at the same position are merged into one launch of the
// table-driven stencil kernels (every problem's arguments in a device
// table), so small problems that could not fill the chip alone run side by
// side.  The merged sequence is captured once in a HIP graph and replayed
// by every run; the temporal depth of the passes and the row-band height of
// the decomposition are chosen by timing candidates on the largest merged
// sweep, re-forward and adjoint passes.
#include "fwi_host.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <new>
#include <vector>

namespace fwi {
namespace batch {

using namespace host;

enum OpKind { OP_FWD = 0, OP_ADJ = 1, OP_CALL = 2, OP_COPY = 3 };

// Schedule position: (phase, a, b, c), compared lexicographically.
struct Key {
    int v[4];
    bool operator<(const Key &o) const {
        for (int k = 0; k < 4; ++k)
            if (v[k] != o.v[k]) return v[k] < o.v[k];
        return false;
    }
    bool operator==(const Key &o) const {
        return v[0] == o.v[0] && v[1] == o.v[1] && v[2] == o.v[2] && v[3] == o.v[3];
    }
};

struct Op {
    Key key;
    OpKind kind;
    int prob;
    FwdStreamArgs fa;
    AdjStreamArgs aa;
    std::function<hipError_t(hipStream_t)> fn;
    std::vector<CopyEntry> cp;     // OP_COPY: device-to-device copies
};

// One executable step of the plan.  A copy step copies the entries of every
// problem's OP_COPY at one schedule position in one launch (table at
// tab_off, prefix sums at boff_off, ctotal floats in all).
struct Step {
    OpKind kind;
    bool tail;
    int depth;                     // temporal depth of a stencil step
    int lev;                       // forward steps: 1 if the entries write every
                                   // level's Ez (segment re-forward), 0 if not
    int nm;
    unsigned nblocks;
    unsigned long long ctotal;     // copy steps: floats copied
    size_t tab_off, boff_off;      // byte offsets in the workspace
    std::function<hipError_t(hipStream_t)> fn;
};

struct Problem {
    fwi_batch_problem u;           // caller's description (pointers)
    Dims d;
    Layout L;
    size_t base;                   // byte offset of this problem's layout
    std::vector<int32_t> src, rec; // host geometry (the caller's arrays may go away)
};

hipError_t ok(int rc) { return rc == FWI_OK ? hipSuccess : hipErrorUnknown; }

// Temporal depth of the passes and row bands of height `rows` (0 = the
// single-problem heuristic for that depth).  The checkpoint interval is a
// multiple of both depths, so the workspace layout does not change.
void set_tiling(Layout &L, int depth, int rows) {
    L.depth = depth;
    if (rows <= 0)
        make_tiling(L.d, L);
    else
        fixed_bands(L, rows, depth);
}

// The operations of one problem's gradient, in its own order, with keys.
void record(int ip, Problem &p, char *ws, std::vector<Op> &ops) {
    const Dims &d = p.d;
    const Layout &L = p.L;
    Ptrs P{ws + p.base, &p.L};
    const fwi_batch_problem u = p.u;
    auto call = [&](Key k, std::function<hipError_t(hipStream_t)> fn) {
        Op o;
        o.key = k;
        o.kind = OP_CALL;
        o.prob = ip;
        o.fn = std::move(fn);
        ops.push_back(std::move(o));
    };
    // E and the full state (H, CPML memories) from (esrc, ssrc) to (edst,
    // sdst), as copy_state and one E copy would do
    auto copies = [&](Key k, float *edst, const float *esrc, const State &sdst,
                      const State &ssrc) {
        const unsigned long long S = (unsigned long long)d.S, f = S * d.plane;
        Op o;
        o.key = k;
        o.kind = OP_COPY;
        o.prob = ip;
        o.cp = {{edst, esrc, f},
                {sdst.Hx, ssrc.Hx, f},
                {sdst.Hy, ssrc.Hy, f},
                {sdst.phx, ssrc.phx, S * d.ys},
                {sdst.phy, ssrc.phy, S * d.xs},
                {sdst.pex, ssrc.pex, S * d.xs},
                {sdst.pey, ssrc.pey, S * d.ys}};
        ops.push_back(std::move(o));
    };
    const size_t field = (size_t)d.S * d.plane;
    const size_t fbytes = field * sizeof(float);
    const int D = L.depth;
    float *Ca = P.f(L.off_Ca), *Cs = P.f(L.off_Cs);
    const State fs[2] = {P.state(L.off_fwd[0], false), P.state(L.off_fwd[1], false)};
    const State as[2] = {P.state(L.off_adj[0], true), P.state(L.off_adj[1], true)};
    float *S1 = P.f(L.off_S1), *S2 = P.f(L.off_S2);

    // phase 0: coefficients of this run's model, zero initial states
    call({{0, 0, 0, 0}}, [=](hipStream_t st) {
        return launch_coefficients(u.eps_r, u.sigma, Ca, Cs, d.NX, d.NY, d.pitch, d.dt, st);
    });
    call({{0, 0, 0, 1}}, [=](hipStream_t st) { return ok(zero_state(fs[0], d, false, st)); });
    call({{0, 0, 0, 2}}, [=](hipStream_t st) { return launch_fill(P.slot(0), field, 0.f, st); });

    // phase 1: forward sweep; E ping-pongs between slots 0 and 1, the full
    // state is copied out at the start of every K-step segment
    FwdStreamArgs a = fwd_args(P);
    a.record = 1;
    int cur = 0, e = 0;
    for (int n0 = 0; n0 < d.nt; n0 += L.K) {
        const int n1 = std::min(d.nt, n0 + L.K);
        const int c = n0 / L.K;
        float *cp = P.f(L.off_ckpt + (size_t)c * L.ckpt_stride);
        const State cst = P.state(L.off_ckpt + (size_t)c * L.ckpt_stride + align_up(fbytes), false);
        copies({{1, n0, 0, 0}}, cp, P.slot(e), cst, fs[cur]);
        for (int n = n0; n < n1; n += D) {
            a.n = n;
            a.nlev = std::min(D, n1 - n);
            a.E_in = P.slot(e);
            e ^= 1;
            a.E_out = P.slot(e);
            a.E_lev = nullptr;
            a.cur = cur;
            a.Hx_in = fs[cur].Hx;
            a.Hy_in = fs[cur].Hy;
            a.Hx_out = fs[cur ^ 1].Hx;
            a.Hy_out = fs[cur ^ 1].Hy;
            Op o;
            o.key = {{1, n, 1, 0}};
            o.kind = OP_FWD;
            o.prob = ip;
            o.fa = a;
            ops.push_back(o);
            cur ^= 1;
        }
    }

    // phase 2: residual and FP64 misfit
    float *trc = P.f(L.off_trc), *res = P.f(L.off_res);
    double *part = reinterpret_cast<double *>(ws + p.base + L.off_mis);
    const size_t ntr = (size_t)d.S * d.nt * d.R;
    call({{2, 0, 0, 0}}, [=](hipStream_t st) {
        return launch_residual_misfit(trc, u.observed, res, ntr, part, u.misfit, st);
    });

    // phase 3: adjoint state and correlation sums to zero
    call({{3, 0, 0, 0}}, [=](hipStream_t st) { return ok(zero_state(as[0], d, true, st)); });
    call({{3, 0, 0, 1}}, [=](hipStream_t st) { return launch_fill(S1, field, 0.f, st); });
    call({{3, 0, 0, 2}}, [=](hipStream_t st) { return launch_fill(S2, field, 0.f, st); });

    // phase 4: segments last first, keyed by their index so that the same
    // time window of every problem lines up: restore the checkpoint, re-run
    // the segment into slots 0..K, then the adjoint through them
    AdjStreamArgs b = adj_args(P);
    int acur = 0;
    constexpr int kSegBase = 1 << 28;
    for (int c = L.ncp - 1; c >= 0; --c) {
        const int n0 = c * L.K, n1 = std::min(d.nt, n0 + L.K);
        const int X = kSegBase - c;
        const float *cp = P.f(L.off_ckpt + (size_t)c * L.ckpt_stride);
        const State cst = P.state(L.off_ckpt + (size_t)c * L.ckpt_stride + align_up(fbytes), false);
        copies({{4, X, 0, 0}}, P.slot(0), cp, fs[0], cst);
        int fcur = 0, j = 0;
        FwdStreamArgs f = fwd_args(P);
        f.record = 0;
        for (int n = n0; n < n1; n += D, ++j) {
            f.n = n;
            f.nlev = std::min(D, n1 - n);
            f.E_in = P.slot(n - n0);
            f.E_lev = P.slot(n + 1 - n0);
            f.E_out = nullptr;
            f.cur = fcur;
            f.Hx_in = fs[fcur].Hx;
            f.Hy_in = fs[fcur].Hy;
            f.Hx_out = fs[fcur ^ 1].Hx;
            f.Hy_out = fs[fcur ^ 1].Hy;
            Op o;
            o.key = {{4, X, 1, j}};
            o.kind = OP_FWD;
            o.prob = ip;
            o.fa = f;
            ops.push_back(o);
            fcur ^= 1;
        }
        j = 0;
        for (int n_top = n1; n_top > n0; n_top -= b.nlev, ++j) {
            // passes start at multiples of the depth, as in the single-problem sweep
            b.nlev = n_top - std::max(n0, (n_top - 1) / D * D);
            b.n_top = n_top;
            b.n_base = n0;
            b.E_lev = P.slot(0);
            b.cur = acur;
            b.L_in = as[acur].E;
            b.LHx_in = as[acur].Hx;
            b.LHy_in = as[acur].Hy;
            b.L_out = as[acur ^ 1].E;
            b.LHx_out = as[acur ^ 1].Hx;
            b.LHy_out = as[acur ^ 1].Hy;
            Op o;
            o.key = {{4, X, 2, j}};
            o.kind = OP_ADJ;
            o.prob = ip;
            o.aa = b;
            ops.push_back(o);
            acur ^= 1;
        }
    }

    // phase 5: shot sums and scaling of the gradients
    call({{5, 0, 0, 0}}, [=](hipStream_t st) {
        return launch_gradient_finalize(u.eps_r, u.sigma, S1, S2, d.S, d.plane, u.grad_eps_r,
                                        u.grad_sigma, d.NX, d.NY, d.pitch, d.dt, st);
    });
}

// Merged, ordered steps; table sizes in bytes (fwd entries, adj entries,
// block offsets) for a plan area at byte offset `area`.
struct Schedule {
    std::vector<Step> steps;
    std::vector<FwdStreamArgs> ftab;
    std::vector<AdjStreamArgs> atab;
    std::vector<unsigned> boff;
    std::vector<CopyEntry> ctab;
    std::vector<unsigned long long> ccum;
    size_t f_off = 0, a_off = 0, b_off = 0, c_off = 0, cc_off = 0, bytes = 0;
    int stencil_launches = 0;
};

size_t area_bytes(size_t nf, size_t na, size_t nb, size_t nc, size_t ncc) {
    return align_up(nf * sizeof(FwdStreamArgs)) + align_up(na * sizeof(AdjStreamArgs)) +
           align_up(nb * sizeof(unsigned)) + align_up(nc * sizeof(CopyEntry)) +
           align_up(ncc * sizeof(unsigned long long));
}

void build_schedule(std::vector<Problem> &probs, char *ws, size_t area, Schedule &S) {
    std::vector<Op> ops;
    for (int i = 0; i < (int)probs.size(); ++i) record(i, probs[i], ws, ops);
    std::stable_sort(ops.begin(), ops.end(), [](const Op &x, const Op &y) { return x.key < y.key; });
    size_t nf = 0, na = 0, nb = 0, nc = 0, ncc = 0;
    for (const Op &o : ops) {
        if (o.kind == OP_FWD) ++nf;
        if (o.kind == OP_ADJ) ++na;
        if (o.kind == OP_COPY) {
            nc += o.cp.size();
            ncc += o.cp.size() + 1;   // upper bound: one extra sum per step
        }
    }
    nb = nf + na + 2 * ops.size();    // upper bound: one offset per entry plus one per
                                      // launch, and every launch holds an entry
    S.f_off = area;
    S.a_off = S.f_off + align_up(nf * sizeof(FwdStreamArgs));
    S.b_off = S.a_off + align_up(na * sizeof(AdjStreamArgs));
    S.c_off = S.b_off + align_up(nb * sizeof(unsigned));
    S.cc_off = S.c_off + align_up(nc * sizeof(CopyEntry));
    S.bytes = area_bytes(nf, na, nb, nc, ncc);
    S.steps.clear();
    S.ftab.clear();
    S.atab.clear();
    S.boff.clear();
    S.ctab.clear();
    S.ccum.clear();
    S.stencil_launches = 0;
    for (size_t i = 0; i < ops.size();) {
        const Op &o = ops[i];
        if (o.kind == OP_CALL) {
            Step s;
            s.kind = OP_CALL;
            s.tail = false;
            s.depth = 0;
            s.lev = 0;
            s.nm = 0;
            s.nblocks = 0;
            s.ctotal = 0;
            s.tab_off = s.boff_off = 0;
            s.fn = o.fn;
            S.steps.push_back(std::move(s));
            ++i;
            continue;
        }
        if (o.kind == OP_COPY) {
            // every problem's copies at this position in one launch
            Step s;
            s.kind = OP_COPY;
            s.tail = false;
            s.depth = 0;
            s.lev = 0;
            s.nm = 0;
            s.nblocks = 0;
            s.ctotal = 0;
            s.tab_off = S.c_off + S.ctab.size() * sizeof(CopyEntry);
            s.boff_off = S.cc_off + S.ccum.size() * sizeof(unsigned long long);
            size_t j = i;
            for (; j < ops.size() && ops[j].kind == OP_COPY && ops[j].key == o.key; ++j)
                for (const CopyEntry &c : ops[j].cp) {
                    S.ccum.push_back(s.ctotal);
                    S.ctab.push_back(c);
                    s.ctotal += c.n;
                    ++s.nm;
                }
            S.ccum.push_back(s.ctotal);
            S.steps.push_back(std::move(s));
            i = j;
            continue;
        }
        size_t j = i;
        while (j < ops.size() && ops[j].kind == o.kind && ops[j].key == o.key) ++j;
        // full-depth and partial passes go to separate launches, and so do
        // forward passes that write every level's Ez and those that do not
        const int depth = o.kind == OP_FWD ? o.fa.tl.depth : o.aa.tl.depth;
        for (int part = 0; part < 4; ++part) {
            const int tail = part & 1, lev = part >> 1;
            if (o.kind == OP_ADJ && lev) continue;
            Step s;
            s.kind = o.kind;
            s.tail = tail != 0;
            s.depth = depth;
            s.lev = lev;
            s.nm = 0;
            s.nblocks = 0;
            s.ctotal = 0;
            s.boff_off = S.b_off + S.boff.size() * sizeof(unsigned);
            s.tab_off = o.kind == OP_FWD ? S.f_off + S.ftab.size() * sizeof(FwdStreamArgs)
                                         : S.a_off + S.atab.size() * sizeof(AdjStreamArgs);
            S.boff.push_back(0);
            for (size_t k = i; k < j; ++k) {
                const Op &q = ops[k];
                const int nlev = q.kind == OP_FWD ? q.fa.nlev : q.aa.nlev;
                if ((nlev < depth) != (tail != 0)) continue;
                if (q.kind == OP_FWD && (q.fa.E_lev != nullptr) != (lev != 0)) continue;
                const Tiling &tl = q.kind == OP_FWD ? q.fa.tl : q.aa.tl;
                const int Sq = q.kind == OP_FWD ? q.fa.S : q.aa.S;
                s.nblocks += stream_blocks(Sq, tl);
                S.boff.push_back(s.nblocks);
                if (q.kind == OP_FWD) S.ftab.push_back(q.fa); else S.atab.push_back(q.aa);
                ++s.nm;
            }
            if (s.nm == 0) {
                S.boff.pop_back();
                continue;
            }
            ++S.stencil_launches;
            S.steps.push_back(std::move(s));
        }
        i = j;
    }
}

hipError_t run_step(const Step &s, char *ws, hipStream_t st) {
    if (s.kind == OP_CALL) return s.fn(st);
    if (s.kind == OP_COPY)
        return launch_copy_table(reinterpret_cast<const CopyEntry *>(ws + s.tab_off),
                                 reinterpret_cast<const unsigned long long *>(ws + s.boff_off),
                                 s.nm, s.ctotal, st);
    const unsigned *boff = reinterpret_cast<const unsigned *>(ws + s.boff_off);
    if (s.kind == OP_FWD)
        return launch_fwd_table(reinterpret_cast<const FwdStreamArgs *>(ws + s.tab_off), boff,
                                s.nm, s.nblocks, s.depth, s.tail, s.lev, st);
    return launch_adj_table(reinterpret_cast<const AdjStreamArgs *>(ws + s.tab_off), boff,
                            s.nm, s.nblocks, s.depth, s.tail, st);
}

int upload_tables(const Schedule &S, char *ws, hipStream_t st) {
    if (!S.ftab.empty())
        FWI_TRY(hipMemcpyAsync(ws + S.f_off, S.ftab.data(), S.ftab.size() * sizeof(FwdStreamArgs),
                               hipMemcpyHostToDevice, st));
    if (!S.atab.empty())
        FWI_TRY(hipMemcpyAsync(ws + S.a_off, S.atab.data(), S.atab.size() * sizeof(AdjStreamArgs),
                               hipMemcpyHostToDevice, st));
    if (!S.boff.empty())
        FWI_TRY(hipMemcpyAsync(ws + S.b_off, S.boff.data(), S.boff.size() * sizeof(unsigned),
                               hipMemcpyHostToDevice, st));
    if (!S.ctab.empty())
        FWI_TRY(hipMemcpyAsync(ws + S.c_off, S.ctab.data(), S.ctab.size() * sizeof(CopyEntry),
                               hipMemcpyHostToDevice, st));
    if (!S.ccum.empty())
        FWI_TRY(hipMemcpyAsync(ws + S.cc_off, S.ccum.data(),
                               S.ccum.size() * sizeof(unsigned long long), hipMemcpyHostToDevice,
                               st));
    FWI_TRY(hipStreamSynchronize(st));
    return FWI_OK;
}

// Problems, common checkpoint interval and layouts; the workspace holds the
// plan tables first, then every problem's layout.
int prepare(int32_t n, const fwi_batch_problem *pp, std::vector<Problem> &probs, int &K) {
    if (n < 1 || !pp) return FWI_EINVAL;
    probs.resize(n);
    double num = 0.0, den = 0.0;
    for (int i = 0; i < n; ++i) {
        Problem &p = probs[i];
        p.u = pp[i];
        if (!p.u.eps_r || !p.u.sigma || !p.u.observed || !p.u.misfit || !p.u.grad_eps_r ||
            !p.u.grad_sigma)
            return FWI_EINVAL;
        int rc = make_dims(&p.u.grid, &p.u.geom, p.d);
        if (rc != FWI_OK) return rc;
        const Dims &d = p.d;
        const double C = 3.0 * d.plane + 2.0 * d.xs + 2.0 * d.ys, E = (double)d.plane;
        num += (double)d.nt * C * d.S;
        den += E * d.S;
        p.src.assign(p.u.geom.src_ij, p.u.geom.src_ij + 2 * (size_t)d.S);
        p.rec.assign(p.u.geom.rec_ij, p.u.geom.rec_ij + 2 * (size_t)d.S * d.R);
        p.u.geom.src_ij = p.src.data();
        p.u.geom.rec_ij = p.rec.data();
    }
    // the interval minimising sum_m ceil(nt_m/K) C_m + (K+1) E_m, a
    // multiple of both temporal depths so that either can run the plan
    K = (int)std::lround(std::sqrt(num / den) / kDepthLarge) * kDepthLarge;
    K = std::max(K, kDepthLarge);
    for (int i = 0; i < n; ++i) {
        int rc = make_layout(probs[i].d, -1, probs[i].L, K, kDepthSmall);
        if (rc != FWI_OK) return rc;
    }
    return FWI_OK;
}

size_t place(std::vector<Problem> &probs, size_t area_end) {
    size_t off = align_up(area_end);
    for (Problem &p : probs) {
        p.base = off;
        off += align_up(p.L.total);
    }
    return off;
}

}  // namespace batch
}  // namespace fwi

using namespace fwi;
using namespace fwi::batch;

struct fwi_batch_plan {
    std::vector<Problem> probs;
    Schedule sched;
    char *ws = nullptr;
    int K = 0;
    int band_rows = 0;
    int depth = kDepthSmall;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    fwi_batch_info info;
};

extern "C" int fwi_batch_workspace_bytes(int32_t n, const fwi_batch_problem *problems,
                                         size_t *bytes) {
    if (!bytes) return FWI_EINVAL;
    std::vector<Problem> probs;
    int K = 0;
    int rc = batch::prepare(n, problems, probs, K);
    if (rc != FWI_OK) return rc;
    for (Problem &p : probs) set_tiling(p.L, kDepthSmall, 0);
    Schedule S;
    // layout offsets do not change the table sizes: count with a null base;
    // depth 4 has the most passes, so its tables are the largest
    place(probs, 0);
    build_schedule(probs, nullptr, 0, S);
    *bytes = place(probs, S.bytes);
    return FWI_OK;
}

extern "C" int fwi_batch_plan_create(int32_t n, const fwi_batch_problem *problems, void *ws,
                                     size_t ws_bytes, int32_t autotune, void *stream,
                                     fwi_batch_plan **out) {
    if (!out) return FWI_EINVAL;
    *out = nullptr;
    if (autotune & ~(FWI_TUNE_BANDS | FWI_TUNE_DEPTH | FWI_BATCH_DEPTH8)) return FWI_EINVAL;
    std::vector<Problem> probs;
    int K = 0;
    int rc = batch::prepare(n, problems, probs, K);
    if (rc != FWI_OK) return rc;
    for (Problem &p : probs) set_tiling(p.L, kDepthSmall, 0);
    Schedule S;
    place(probs, 0);
    build_schedule(probs, nullptr, 0, S);
    const size_t need = place(probs, S.bytes);
    if (!ws || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0 || ws_bytes < need)
        return FWI_ENOMEM;
    fwi_batch_plan *plan = new (std::nothrow) fwi_batch_plan;
    if (!plan) return FWI_ENOMEM;
    hipStream_t st = static_cast<hipStream_t>(stream);
    plan->ws = static_cast<char *>(ws);
    plan->K = K;
    std::memset(&plan->info, 0, sizeof(plan->info));
    char *w = plan->ws;
    auto fail = [&](int code) {
        delete plan;
        return code;
    };

    // geometry, cold arguments and CPML profiles of every problem (once)
    auto upload_all = [&]() -> int {
        for (Problem &p : probs) {
            Ptrs P{w + p.base, &p.L};
            const StreamCold cold = make_cold(P, &p.u.geom, P.f(p.L.off_trc), P.f(p.L.off_res),
                                              nullptr);
            int r = upload_geometry(P, &p.u.geom, cold, st);
            if (r != FWI_OK) return r;
        }
        return FWI_OK;
    };
    rc = upload_all();
    if (rc != FWI_OK) return fail(rc);
    for (Problem &p : probs) {
        Ptrs P{w + p.base, &p.L};
        if (launch_profiles(p.d, P.prof(), st) != hipSuccess) return fail(FWI_EHIP);
    }

    // candidates: temporal depth x row-band height
    std::vector<int> depths, heights;
    if (autotune & FWI_TUNE_DEPTH) {
        depths = {kDepthSmall, kDepthLarge};
    } else {
        depths = {(autotune & FWI_BATCH_DEPTH8) ? kDepthLarge : kDepthSmall};
    }
    if (autotune & FWI_TUNE_BANDS)
        heights = {0, 32, 64, 128, 256, 512, 1 << 20};
    else
        heights = {0};
    int depth = depths[0], rows = heights[0];
    if (depths.size() * heights.size() > 1) {
        // time, for every candidate, the largest merged full-depth launch of
        // each pass kind (best of 3 each): the forward sweep, the segment
        // re-forward and the adjoint.  A gradient runs one of each per
        // `depth` steps, so the cost per step is (sweep + re-forward +
        // adjoint) / depth.  The largest launches are those where every
        // problem takes part; the first adjoint launches hold only the
        // longest problems.  The re-forward and adjoint passes run on
        // whatever state the workspace holds (all of it allocated); their
        // time does not depend on the values, and every run of the plan
        // clears that state first.
        double best = 1e300;
        hipEvent_t e0, e1;
        if (hipEventCreate(&e0) != hipSuccess) return fail(FWI_EHIP);
        if (hipEventCreate(&e1) != hipSuccess) {
            (void)hipEventDestroy(e0);
            return fail(FWI_EHIP);
        }
        auto time_step = [&](const Step &s, float &ms_min) -> int {
            ms_min = 1e30f;
            for (int rep = 0; rep < 3; ++rep) {
                if (hipEventRecord(e0, st) != hipSuccess || run_step(s, w, st) != hipSuccess ||
                    hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
                    return FWI_EHIP;
                float ms = 0.f;
                if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return FWI_EHIP;
                ms_min = std::min(ms_min, ms);
            }
            return FWI_OK;
        };
        int tuned = 0;
        for (int dep : depths) {
            for (int h : heights) {
                for (Problem &p : probs) set_tiling(p.L, dep, h);
                rc = upload_all();
                if (rc != FWI_OK) break;
                build_schedule(probs, w, 0, S);
                rc = upload_tables(S, w, st);
                if (rc != FWI_OK) break;
                // run the set-up steps once so the first pass reads valid state
                size_t first = 0;
                while (first < S.steps.size() &&
                       (S.steps[first].kind == OP_CALL || S.steps[first].kind == OP_COPY)) {
                    if (run_step(S.steps[first], w, st) != hipSuccess) rc = FWI_EHIP;
                    ++first;
                }
                // largest full-depth launch of a kind (forward: of a
                // level-store choice), else the largest partial one
                auto largest = [&](OpKind kind, int lev) {
                    size_t best_k = S.steps.size();
                    for (size_t k = first; k < S.steps.size(); ++k) {
                        const Step &q = S.steps[k];
                        if (q.kind != kind || (kind == OP_FWD && q.lev != lev)) continue;
                        if (best_k == S.steps.size()) {
                            best_k = k;
                            continue;
                        }
                        const Step &b = S.steps[best_k];
                        if ((b.tail && !q.tail) ||
                            (b.tail == q.tail && q.nblocks > b.nblocks))
                            best_k = k;
                    }
                    return best_k;
                };
                const size_t fsw = largest(OP_FWD, 0), fre = largest(OP_FWD, 1),
                             fadj = largest(OP_ADJ, 0);
                if (rc != FWI_OK || fsw >= S.steps.size() || fadj >= S.steps.size()) {
                    rc = rc == FWI_OK ? FWI_EHIP : rc;
                    break;
                }
                float tf = 0.f, tr = 0.f, ta = 0.f;
                rc = time_step(S.steps[fsw], tf);
                if (rc == FWI_OK && fre < S.steps.size()) rc = time_step(S.steps[fre], tr);
                else tr = tf;
                if (rc == FWI_OK) rc = time_step(S.steps[fadj], ta);
                if (rc != FWI_OK) break;
                const double cost = ((double)tf + tr + ta) / dep;
                if (tuned < FWI_BATCH_MAX_TUNE) {
                    plan->info.tune_depth[tuned] = dep;
                    plan->info.tune_rows[tuned] = h;
                    plan->info.tune_ms[tuned] = cost;
                    ++tuned;
                }
                if (cost < best * 0.98) {
                    best = cost;
                    depth = dep;
                    rows = h;
                }
            }
            if (rc != FWI_OK) break;
        }
        plan->info.ntune = tuned;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (rc != FWI_OK) return fail(rc);
    }
    for (Problem &p : probs) set_tiling(p.L, depth, rows);
    rc = upload_all();
    if (rc != FWI_OK) return fail(rc);
    build_schedule(probs, w, 0, S);
    rc = upload_tables(S, w, st);
    if (rc != FWI_OK) return fail(rc);

    // capture the whole sequence once, on a private stream (the caller's may
    // be the null stream, which cannot be captured); runs launch the graph
    // on the caller's stream
    bool captured = false;
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) == hipSuccess) {
        if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess) {
            hipError_t e = hipSuccess;
            for (const Step &s : S.steps) {
                e = run_step(s, w, cs);
                if (e != hipSuccess) break;
            }
            hipGraph_t g = nullptr;
            const hipError_t ee = hipStreamEndCapture(cs, &g);
            if (e == hipSuccess && ee == hipSuccess && g &&
                hipGraphInstantiate(&plan->exec, g, nullptr, nullptr, 0) == hipSuccess) {
                plan->graph = g;
                captured = true;
            } else if (g) {
                (void)hipGraphDestroy(g);
            }
        }
        (void)hipStreamDestroy(cs);
    }
    (void)hipGetLastError();
    plan->probs = std::move(probs);
    plan->sched = std::move(S);
    plan->band_rows = rows;
    plan->depth = depth;
    plan->info.nproblems = n;
    plan->info.checkpoint_interval = K;
    plan->info.band_rows = rows;
    plan->info.depth = depth;
    plan->info.steps = (int32_t)plan->sched.steps.size();
    plan->info.stencil_launches = plan->sched.stencil_launches;
    plan->info.graph = captured ? 1 : 0;
    *out = plan;
    return FWI_OK;
}

extern "C" int fwi_batch_plan_run(fwi_batch_plan *plan, int32_t use_graph, void *stream) {
    if (!plan) return FWI_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (use_graph && plan->exec) {
        FWI_TRY(hipGraphLaunch(plan->exec, st));
        return FWI_OK;
    }
    for (const Step &s : plan->sched.steps) FWI_TRY(run_step(s, plan->ws, st));
    return FWI_OK;
}

extern "C" int fwi_batch_plan_info(const fwi_batch_plan *plan, fwi_batch_info *info) {
    if (!plan || !info) return FWI_EINVAL;
    *info = plan->info;
    return FWI_OK;
}

extern "C" void fwi_batch_plan_destroy(fwi_batch_plan *plan) {
    if (!plan) return;
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    delete plan;
}
