// Host side of the FWI library: argument validation (pure host code, runs
// before any HIP call), workspace layout, and the time loops of the forward
// sweep (Algorithm 1), the adjoint sweep (Algorithm 2) and the full gradient
// evaluation.  Paper: arXiv 2506.20513, Secs. 2.1 and 3.3.
#include "fwi_host.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>
#include <vector>

namespace fwi {
namespace host {


bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Grid checks: shapes, spacings, CFL bound (Eq. (11) with c = c0, the fastest
// speed any model with eps_r >= 1 can have), CPML parameters.
int check_grid(const fwi_grid *g) {
    if (!g) return FWI_EINVAL;
    if (g->nx < 1 || g->ny < 1 || g->npml < 0 || g->nt < 1) return FWI_EINVAL;
    const int64_t NX = (int64_t)g->nx + 2 * (int64_t)g->npml;
    const int64_t NY = (int64_t)g->ny + 2 * (int64_t)g->npml;
    if (NX < 3 || NY < 3 || NX > (1 << 20) || NY > (1 << 20)) return FWI_EINVAL;
    // the stencil kernels address one shot's plane with 32-bit byte offsets
    if ((NX + 63) / 64 * 64 * NY >= ((int64_t)1 << 30)) return FWI_EINVAL;
    if (!finite_pos(g->dx) || !finite_pos(g->dy) || !finite_pos(g->dt)) return FWI_EINVAL;
    if (g->cpml_order < 1 || g->cpml_order > 16) return FWI_EINVAL;
    if (!std::isfinite(g->cpml_sigma_scale) || g->cpml_sigma_scale < 0.0) return FWI_EINVAL;
    if (!std::isfinite(g->cpml_kappa_max) || g->cpml_kappa_max < 1.0) return FWI_EINVAL;
    if (!std::isfinite(g->cpml_alpha_max) || g->cpml_alpha_max < 0.0) return FWI_EINVAL;
    const double bound = 1.0 / (kC0 * std::sqrt(1.0 / (g->dx * g->dx) + 1.0 / (g->dy * g->dy)));
    if (g->dt > bound * (1.0 + 1e-12)) return FWI_ECFL;
    return FWI_OK;
}

bool inside(int i, int j, const Dims &d) {
    const int lo_i = std::max(d.npml, 1), hi_i = std::min(d.NX - 1 - d.npml, d.NX - 2);
    const int lo_j = std::max(d.npml, 1), hi_j = std::min(d.NY - 1 - d.npml, d.NY - 2);
    return i >= lo_i && i <= hi_i && j >= lo_j && j <= hi_j;
}

int check_geom(const fwi_geom *g, Dims &d) {
    if (!g) return FWI_EINVAL;
    if (g->nshots < 1 || g->nrec < 1) return FWI_EINVAL;
    if ((int64_t)g->nshots * g->nrec > (1 << 28)) return FWI_EINVAL;
    if (!g->src_ij || !g->rec_ij || !g->wavelet) return FWI_EINVAL;
    d.S = g->nshots;
    d.R = g->nrec;
    for (int s = 0; s < d.S; ++s)
        if (!inside(g->src_ij[2 * s], g->src_ij[2 * s + 1], d)) return FWI_EGEOM;
    const size_t nr = (size_t)d.S * d.R;
    for (size_t t = 0; t < nr; ++t)
        if (!inside(g->rec_ij[2 * t], g->rec_ij[2 * t + 1], d)) return FWI_EGEOM;
    return FWI_OK;
}

int make_dims(const fwi_grid *grid, const fwi_geom *geom, Dims &d) {
    int st = check_grid(grid);
    if (st != FWI_OK) return st;
    d.npml = grid->npml;
    d.nt = grid->nt;
    d.NX = grid->nx + 2 * grid->npml;
    d.NY = grid->ny + 2 * grid->npml;
    d.pitch = (d.NX + 63) / 64 * 64;
    d.W = 2 * d.npml + 1;
    d.Hs = 2 * d.npml + 1;
    d.plane = (size_t)d.NY * d.pitch;
    d.xs = (size_t)d.NY * d.W;
    d.ys = (size_t)d.Hs * d.pitch;
    d.dx = grid->dx;
    d.dy = grid->dy;
    d.dt = grid->dt;
    d.cpml_order = grid->cpml_order;
    d.cpml_sigma_scale = grid->cpml_sigma_scale;
    d.cpml_kappa_max = grid->cpml_kappa_max;
    d.cpml_alpha_max = grid->cpml_alpha_max;
    return check_geom(geom, d);
}

// Temporal depth of a single problem's streaming passes (see kDepthLarge).
int stream_depth(const Dims &d) {
    return (long long)d.NX * d.NY >= kDepthLargeCells ? kDepthLarge : kDepthSmall;
}

// Checkpoint interval minimising checkpoints + segment buffer,
// ceil(nt/K) * C + (K+1) * E with C one full state and E one Ez slot, rounded
// to a multiple of the temporal depth so segments split into full passes.
int choose_k(const Dims &d, int depth) {
    const double C = 3.0 * d.plane + 2.0 * d.xs + 2.0 * d.ys;
    const double E = (double)d.plane;
    const double k = std::sqrt((double)d.nt * C / E);
    int K = (int)std::lround(k / depth) * depth;
    K = std::max(K, depth);
    return std::max(1, std::min(K, d.nt));
}

// Streaming decomposition: x strips of 64 - 2K output columns, and row bands
// chosen so that the waves fill whole rounds of the chip: each band costs 2K
// rows of start-up on top of its own rows, and a last partial round of waves
// leaves SIMDs idle; pick the band count with the least estimated time.  The
// waves of one round do not all finish together, so the idle part of the
// last round counts half (fitted to band-count sweeps on 2088x1064 x 64
// shots, best at 4 bands for the forward kernel and 2 for the adjoint, and
// on 552x296 x 24 shots, best at 17 for both).  `waves` is the kernel's
// resident waves per SIMD.  A launch that shares the chip with the launches
// of `groups` - 1 other shot groups counts 1/groups of the slots: fewer,
// taller bands, whose pipeline starts and last rounds the other groups'
// waves overlap (on 552x296 x 24 shots in three groups 0.157 against
// 0.164 s per gradient; on 2088x1064 x 64 shots 4.86 against 4.94 s).
int pick_bands(const Dims &d, int K, int nstrip, double waves, int *bands, int groups) {
    const int max_bands = 63;
    const double slots = 256.0 * 4.0 * waves / groups;   // 256 CUs x 4 SIMDs
    const double per_band = (double)d.S * nstrip;
    int best = 1;
    double best_t = 1e300;
    for (int nb = 1; nb <= max_bands && nb <= (d.NY + 2 * K - 1) / (2 * K); ++nb) {
        const int h = (d.NY + nb - 1) / nb;
        const double r = per_band * nb / slots;
        const double rounds = r <= 1.0 ? 1.0 : r + 0.5 * (std::ceil(r) - r);
        const double t = rounds * (h + 2.0 * K);
        if (t < best_t * 0.999) {
            best_t = t;
            best = nb;
        }
    }
    const int h = (d.NY + best - 1) / best;
    int nb = 0;
    for (int y = 0; y < d.NY; y += h) bands[nb++] = y;
    bands[nb] = d.NY;
    return nb;
}

// Resident waves per SIMD of the stencil kernels (512 VGPRs per SIMD lane):
// the forward kernels need 75-123 VGPRs (4 waves at depth 8; at depth 4 the
// estimate stays at 4, which the sweeps above favour), the depth-8 adjoint
// 165 (3 waves).
constexpr double kFwdWaves = 4.0;
double adj_waves(int depth) { return depth == kDepthLarge ? 3.0 : 4.0; }

void make_tiling(const Dims &d, Layout &L, int groups) {
    static_assert(sizeof(L.bands) / sizeof(int) == 64 && sizeof(L.abands) / sizeof(int) == 64,
                  "band tables hold 63 bands");
    const int K = L.depth, OW = 64 - 2 * K;
    L.nstrip = (d.NX + OW - 1) / OW;
    L.nband = pick_bands(d, K, L.nstrip, kFwdWaves, L.bands, groups);
    L.naband = pick_bands(d, K, L.nstrip, adj_waves(K), L.abands, groups);
}

void fixed_bands(Layout &L, int rows, int depth) {
    const int OW = 64 - 2 * depth;
    const int max_bands = (int)(sizeof(L.bands) / sizeof(int)) - 1;
    L.nstrip = (L.d.NX + OW - 1) / OW;
    const int h = std::max(rows, (L.d.NY + max_bands - 1) / max_bands);
    int nb = 0;
    for (int y = 0; y < L.d.NY; y += h) {
        L.bands[nb] = L.abands[nb] = y;
        ++nb;
    }
    L.nband = L.naband = nb;
    L.bands[nb] = L.abands[nb] = L.d.NY;
}

// Workspace layout for a mode (FWI_SAVE_* or -1 = fwi_gradient).  With
// `shared` (gradient mode only), the layout is one shot group's: it starts
// at byte `start`, and its coefficients, profiles, imaging sums, traces,
// residual and reduction partials are those of `shared` (the sums, traces
// and residual at the group's first shot s0).
int make_layout(const Dims &d, int mode, Layout &L, int k, int depth, size_t start,
                const Layout *shared, int s0) {
    if (mode != FWI_SAVE_NONE && mode != FWI_SAVE_CHECKPOINT &&
        mode != FWI_SAVE_HISTORY && mode != -1)
        return FWI_EINVAL;
    if (shared && mode != -1) return FWI_EINVAL;
    L.d = d;
    L.mode = mode;
    L.depth = depth > 0 ? depth : stream_depth(d);
    const size_t S = (size_t)d.S;
    const size_t field = S * d.plane * sizeof(float);
    const size_t xs = S * d.xs * sizeof(float), ys = S * d.ys * sizeof(float);
    size_t off = start;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align_up(bytes);
        return o;
    };
    if (shared) {
        L.off_Ca = shared->off_Ca;
        L.off_Cs = shared->off_Cs;
        L.off_prof = shared->off_prof;
    } else {
        L.off_Ca = take(d.plane * sizeof(float));
        L.off_Cs = take(d.plane * sizeof(float));
        L.off_prof = take((size_t)6 * (d.NX + d.NY) * sizeof(float));
    }
    L.off_src = take(S * 2 * sizeof(int));
    L.off_rrow = take(S * (d.NY + 1) * sizeof(int));
    L.off_rcol = take(S * d.R * sizeof(int));
    L.off_ridx = take(S * d.R * sizeof(int));
    L.off_rspan = take(S * 2 * sizeof(int));
    L.off_bands = take(sizeof(L.bands));
    L.off_abands = take(sizeof(L.abands));
    L.off_cold = take(sizeof(StreamCold));
    L.state_bytes = align_up(field) * 2 + align_up(xs) * 2 + align_up(ys) * 2;
    L.off_fwd[0] = take(L.state_bytes);
    L.off_fwd[1] = take(L.state_bytes);
    L.K = 0;
    L.ncp = 0;
    L.ckpt_stride = 0;
    L.off_ckpt = 0;
    if (mode == FWI_SAVE_NONE) {
        L.nslots = 2;
    } else if (mode == FWI_SAVE_HISTORY) {
        L.nslots = d.nt + 1;
    } else {
        L.K = k > 0 ? std::min(k, d.nt) : choose_k(d, L.depth);
        L.ncp = (d.nt + L.K - 1) / L.K;
        L.nslots = L.K + 1;
    }
    if ((double)L.nslots * (double)field > 1e15) return FWI_EINVAL;
    L.off_slots = take((size_t)L.nslots * field);
    if (L.ncp > 0) {
        L.ckpt_stride = align_up(field) + L.state_bytes;
        L.off_ckpt = take((size_t)L.ncp * L.ckpt_stride);
    }
    L.off_adj[0] = L.off_adj[1] = L.off_S1 = L.off_S2 = 0;
    if (mode != FWI_SAVE_NONE) {
        L.off_adj[0] = take(align_up(field) + L.state_bytes);
        L.off_adj[1] = take(align_up(field) + L.state_bytes);
        if (!shared) {
            L.off_S1 = take(field);
            L.off_S2 = take(field);
        }
    }
    L.off_res = L.off_trc = L.off_mis = 0;
    if (shared) {
        const size_t sp = (size_t)s0 * d.plane * sizeof(float);
        const size_t st = (size_t)s0 * d.R * (size_t)d.nt * sizeof(float);
        L.off_S1 = shared->off_S1 + sp;
        L.off_S2 = shared->off_S2 + sp;
        L.off_res = shared->off_res + st;
        L.off_trc = shared->off_trc + st;
        L.off_mis = shared->off_mis;
        L.off_chk = shared->off_chk;
    } else {
        if (mode == -1) {
            const size_t tr = S * d.R * (size_t)d.nt * sizeof(float);
            L.off_res = take(tr);
            L.off_trc = take(tr);
            L.off_mis = take(kMisfitBlocks * sizeof(double));
        }
        L.off_chk = take(kMisfitBlocks * sizeof(double) + sizeof(int));
    }
    L.total = off;
    make_tiling(d, L);
    return FWI_OK;
}

// The gradient's shots in G groups (shots s0[g] .. s0[g+1]-1) that run
// concurrently, each on its own stream: the arrays that every group reads
// (coefficients, profiles) or that a step after the groups reads across all
// shots (imaging sums, traces, residual, reduction partials) once, laid out
// as a full layout would, then each group's own layout (geometry tables,
// states, Ez slots, checkpoints).  Every shot's arithmetic is the same as in
// a single group, so the results are identical bit for bit.
int make_group_layout(const Dims &d, int G, GroupLayout &GL) {
    if (G < 1 || G > kMaxShotGroups || G > d.S) return FWI_EINVAL;
    GL.G = G;
    Layout &sh = GL.shared;
    sh = Layout{};
    sh.d = d;
    sh.mode = -1;
    const size_t S = (size_t)d.S;
    const size_t field = S * d.plane * sizeof(float);
    const size_t tr = S * d.R * (size_t)d.nt * sizeof(float);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align_up(bytes);
        return o;
    };
    sh.off_Ca = take(d.plane * sizeof(float));
    sh.off_Cs = take(d.plane * sizeof(float));
    sh.off_prof = take((size_t)6 * (d.NX + d.NY) * sizeof(float));
    sh.off_S1 = take(field);
    sh.off_S2 = take(field);
    sh.off_res = take(tr);
    sh.off_trc = take(tr);
    sh.off_mis = take(kMisfitBlocks * sizeof(double));
    sh.off_chk = take(kMisfitBlocks * sizeof(double) + sizeof(int));
    for (int g = 0; g <= G; ++g) GL.s0[g] = (int)((long long)g * d.S / G);
    for (int g = 0; g < G; ++g) {
        Dims dg = d;
        dg.S = GL.s0[g + 1] - GL.s0[g];
        const int rc = make_layout(dg, -1, GL.grp[g], 0, 0, off, &sh, GL.s0[g]);
        if (rc != FWI_OK) return rc;
        make_tiling(dg, GL.grp[g], G);
        off = GL.grp[g].total;
    }
    sh.total = off;
    GL.total = off;
    return FWI_OK;
}

// Shot groups of a gradient call: with 16 or more shots, one group per 6
// shots up to four; one group otherwise.  The groups' launches fill each
// other's last, partial rounds of waves and hide each other's pipeline
// starts.  Group 0 runs on the caller's stream, so four groups use four
// streams, as many as the hardware queues a process gets by default (with
// every group on a new stream, the fifth stream made four groups slower than
// three).  Measured (one group -> two -> three -> four): 2088 x 1064 cells,
// 64 shots: 5.60 -> 4.97 -> 4.87 -> 4.80 s; 552 x 296 cells, 24 shots:
// 0.175 -> 0.177 -> 0.149 -> 0.147 s.
int auto_shot_groups(const Dims &d) {
    return d.S >= 16 ? std::min(kMaxShotGroups, d.S / 6) : 1;
}

// Gradient workspace: enough for one group and for every group count up to
// kMaxShotGroups (the groups add only small per-group tables).
int gradient_workspace(const Dims &d, size_t &bytes) {
    Layout L;
    int rc = make_layout(d, -1, L);
    if (rc != FWI_OK) return rc;
    bytes = L.total;
    for (int G = 2; G <= kMaxShotGroups && G <= d.S; ++G) {
        GroupLayout GL;
        rc = make_group_layout(d, G, GL);
        if (rc != FWI_OK) return rc;
        bytes = std::max(bytes, GL.total);
    }
    return FWI_OK;
}

// End-of-call finiteness check of a call's outputs (FP64 sums of squares of
// up to two float arrays and an optional device double): waits for the
// stream and returns FWI_ENONFINITE if any of them holds a NaN or infinity.
int check_finite(const Ptrs &P, const float *a, size_t na, const float *b, size_t nb,
                 const double *scalar, hipStream_t st) {
    double *partials = reinterpret_cast<double *>(P.base + P.L->off_chk);
    int *flag = reinterpret_cast<int *>(partials + kMisfitBlocks);
    FWI_TRY(launch_finite_check(a, na, b, nb, scalar, partials, flag, st));
    int h = 0;
    FWI_TRY(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    FWI_TRY(hipStreamSynchronize(st));
    return h ? FWI_ENONFINITE : FWI_OK;
}

// Geometry to the device: sources, and per shot the receivers sorted by
// (row, column) - stable in receiver index, so receivers sharing a cell stay
// in index order - with a row CSR.
int upload_geometry(const Ptrs &P, const fwi_geom *g, const StreamCold &cold,
                    hipStream_t st) {
    const Dims &d = P.L->d;
    const size_t S = d.S, R = d.R, NY = d.NY;
    std::vector<int> rrow(S * (NY + 1)), rcol(S * R), ridx(S * R), rspan(S * 2);
    for (size_t s = 0; s < S; ++s) {
        const int32_t *rc = g->rec_ij + 2 * s * R;
        int *o = ridx.data() + s * R;
        std::iota(o, o + R, 0);
        std::stable_sort(o, o + R, [&](int a, int b) {
            const int64_t ka = (int64_t)rc[2 * a + 1] * d.NX + rc[2 * a];
            const int64_t kb = (int64_t)rc[2 * b + 1] * d.NX + rc[2 * b];
            return ka < kb;
        });
        int *rr = rrow.data() + s * (NY + 1);
        size_t q = 0;
        for (size_t j = 0; j <= NY; ++j) {
            while (q < R && (size_t)rc[2 * o[q] + 1] < j) ++q;
            rr[j] = (int)q;
        }
        for (size_t k = 0; k < R; ++k) rcol[s * R + k] = rc[2 * o[k]];
        rspan[2 * s] = rc[2 * o[0] + 1];
        rspan[2 * s + 1] = rc[2 * o[R - 1] + 1];
    }
    FWI_TRY(hipMemcpyAsync(P.i(P.L->off_src), g->src_ij, S * 2 * sizeof(int),
                           hipMemcpyHostToDevice, st));
    FWI_TRY(hipMemcpyAsync(P.i(P.L->off_rrow), rrow.data(), rrow.size() * sizeof(int),
                           hipMemcpyHostToDevice, st));
    FWI_TRY(hipMemcpyAsync(P.i(P.L->off_rcol), rcol.data(), rcol.size() * sizeof(int),
                           hipMemcpyHostToDevice, st));
    FWI_TRY(hipMemcpyAsync(P.i(P.L->off_ridx), ridx.data(), ridx.size() * sizeof(int),
                           hipMemcpyHostToDevice, st));
    FWI_TRY(hipMemcpyAsync(P.i(P.L->off_rspan), rspan.data(), rspan.size() * sizeof(int),
                           hipMemcpyHostToDevice, st));
    FWI_TRY(hipMemcpyAsync(P.i(P.L->off_bands), P.L->bands, sizeof(P.L->bands),
                           hipMemcpyHostToDevice, st));
    FWI_TRY(hipMemcpyAsync(P.i(P.L->off_abands), P.L->abands, sizeof(P.L->abands),
                           hipMemcpyHostToDevice, st));
    FWI_TRY(hipMemcpyAsync(P.base + P.L->off_cold, &cold, sizeof(StreamCold),
                           hipMemcpyHostToDevice, st));
    // pageable host sources: make sure the copies consumed them before the
    // vectors go out of scope
    FWI_TRY(hipStreamSynchronize(st));
    return FWI_OK;
}

int zero_state(const State &s, const Dims &d, bool with_e, hipStream_t st) {
    const size_t S = d.S;
    if (with_e) FWI_TRY(launch_fill(s.E, S * d.plane, 0.f, st));
    FWI_TRY(launch_fill(s.Hx, S * d.plane, 0.f, st));
    FWI_TRY(launch_fill(s.Hy, S * d.plane, 0.f, st));
    FWI_TRY(launch_fill(s.phx, S * d.ys, 0.f, st));
    FWI_TRY(launch_fill(s.phy, S * d.xs, 0.f, st));
    FWI_TRY(launch_fill(s.pex, S * d.xs, 0.f, st));
    FWI_TRY(launch_fill(s.pey, S * d.ys, 0.f, st));
    return FWI_OK;
}

int copy_state(const State &dst, const State &src, const Dims &d, hipStream_t st) {
    const size_t S = d.S;
    const size_t f = S * d.plane * sizeof(float);
    FWI_TRY(hipMemcpyAsync(dst.Hx, src.Hx, f, hipMemcpyDeviceToDevice, st));
    FWI_TRY(hipMemcpyAsync(dst.Hy, src.Hy, f, hipMemcpyDeviceToDevice, st));
    FWI_TRY(hipMemcpyAsync(dst.phx, src.phx, S * d.ys * sizeof(float), hipMemcpyDeviceToDevice, st));
    FWI_TRY(hipMemcpyAsync(dst.phy, src.phy, S * d.xs * sizeof(float), hipMemcpyDeviceToDevice, st));
    FWI_TRY(hipMemcpyAsync(dst.pex, src.pex, S * d.xs * sizeof(float), hipMemcpyDeviceToDevice, st));
    FWI_TRY(hipMemcpyAsync(dst.pey, src.pey, S * d.ys * sizeof(float), hipMemcpyDeviceToDevice, st));
    return FWI_OK;
}

Tiling tiling(const Ptrs &P) {
    const Layout &L = *P.L;
    Tiling t;
    t.bands = P.i(L.off_bands);
    t.nstrip = L.nstrip;
    t.nband = L.nband;
    t.depth = L.depth;
    return t;
}

Tiling tiling_adj(const Ptrs &P) {
    Tiling t = tiling(P);
    t.bands = P.i(P.L->off_abands);
    t.nband = P.L->naband;
    return t;
}

// The per-call cold arguments of the stencil kernels (see StreamCold).
StreamCold make_cold(const Ptrs &P, const fwi_geom *g, float *traces,
                     const float *residual, float *src_adjoint) {
    const Layout &L = *P.L;
    StreamCold c;
    c.p = P.prof();
    c.fs[0] = P.state(L.off_fwd[0], false);
    c.fs[1] = P.state(L.off_fwd[1], false);
    if (L.mode != FWI_SAVE_NONE) {
        c.as[0] = P.state(L.off_adj[0], true);
        c.as[1] = P.state(L.off_adj[1], true);
    } else {
        c.as[0] = c.as[1] = State{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    }
    c.g.src_ij = P.i(L.off_src);
    c.g.wavelet = g->wavelet;
    c.g.rrow = P.i(L.off_rrow);
    c.g.rcol = P.i(L.off_rcol);
    c.g.ridx = P.i(L.off_ridx);
    c.g.rspan = P.i(L.off_rspan);
    c.traces = traces;
    c.residual = residual;
    c.src_adjoint = src_adjoint;
    return c;
}

FwdStreamArgs fwd_args(const Ptrs &P) {
    const Layout &L = *P.L;
    const Dims &d = L.d;
    FwdStreamArgs a;
    a.NX = d.NX; a.NY = d.NY; a.npml = d.npml; a.pitch = d.pitch;
    a.W = d.W; a.S = d.S; a.R = d.R; a.nt = d.nt;
    a.n = 0; a.nlev = 0; a.cur = 0; a.record = 0;
    a.tl = tiling(P);
    a.plane = d.plane; a.xs = d.xs; a.ys = d.ys;
    a.lev_stride = (size_t)d.S * d.plane;
    a.ch = (float)(d.dt / kMu0);
    a.rdx = (float)(1.0 / d.dx);
    a.rdy = (float)(1.0 / d.dy);
    a.src_scale = (float)(1.0 / (d.dx * d.dy));
    a.Ca = P.f(L.off_Ca);
    a.Cs = P.f(L.off_Cs);
    a.E_in = nullptr; a.E_out = nullptr; a.E_lev = nullptr;
    a.Hx_in = a.Hy_in = nullptr;
    a.Hx_out = a.Hy_out = nullptr;
    a.cold = reinterpret_cast<const StreamCold *>(P.base + L.off_cold);
    return a;
}

AdjStreamArgs adj_args(const Ptrs &P) {
    const Layout &L = *P.L;
    const Dims &d = L.d;
    AdjStreamArgs a;
    a.NX = d.NX; a.NY = d.NY; a.npml = d.npml; a.pitch = d.pitch;
    a.W = d.W; a.S = d.S; a.R = d.R; a.nt = d.nt;
    a.n_top = a.n_base = a.nlev = a.cur = 0;
    a.tl = tiling_adj(P);
    a.plane = d.plane; a.xs = d.xs; a.ys = d.ys;
    a.lev_stride = (size_t)d.S * d.plane;
    a.ch = (float)(d.dt / kMu0);
    a.rdx = (float)(1.0 / d.dx);
    a.rdy = (float)(1.0 / d.dy);
    a.src_scale = (float)(1.0 / (d.dx * d.dy));
    a.Ca = P.f(L.off_Ca);
    a.Cs = P.f(L.off_Cs);
    a.E_lev = nullptr;
    a.L_in = a.LHx_in = a.LHy_in = nullptr;
    a.L_out = a.LHx_out = a.LHy_out = nullptr;
    a.S1 = L.off_S1 ? P.f(L.off_S1) : nullptr;
    a.S2 = L.off_S2 ? P.f(L.off_S2) : nullptr;
    a.cold = reinterpret_cast<const StreamCold *>(P.base + L.off_cold);
    return a;
}

}  // namespace host

namespace {

using namespace host;

// Optional per-kernel timing with HIP events on the call's stream.  The
// forward kernel is timed as two kinds: passes that write only the final
// state (the forward sweep, k_fwd<K, *, 0>) and passes that write every
// level's Ez (the segment re-forward, k_fwd<K, *, 1>).
enum Kind { K_FWD_SWEEP = 0, K_FWD_REFWD = 1, K_ADJ = 2, K_NKINDS = 3 };
const char *const kKindName[K_NKINDS] = {"k_fwd_sweep", "k_fwd_reforward", "k_adj"};

struct Timer {
    fwi_timing *t = nullptr;
    hipStream_t st = nullptr;
    int launches[K_NKINDS] = {0, 0, 0};
    double updates[K_NKINDS] = {0, 0, 0};
    struct Rec { int kind; hipEvent_t a, b; };
    std::vector<Rec> recs;
    bool failed = false;

    // Launch `fn` (returning hipError_t), bracketed by events when sampled.
    template <class F>
    hipError_t run(int kind, double cell_updates, F fn) {
        updates[kind] += cell_updates;
        const int idx = launches[kind]++;
        if (!t || idx % t->sample_every != 0 || failed) return fn();
        Rec r{kind, nullptr, nullptr};
        if (hipEventCreate(&r.a) != hipSuccess) { failed = true; return fn(); }
        if (hipEventCreate(&r.b) != hipSuccess) {
            (void)hipEventDestroy(r.a);
            failed = true;
            return fn();
        }
        hipError_t e = hipEventRecord(r.a, st);
        if (e == hipSuccess) e = fn();
        if (e == hipSuccess) e = hipEventRecord(r.b, st);
        recs.push_back(r);
        return e;
    }

    // Wait for the stream, add the sampled launches' durations to sum / cnt
    // and release the events.
    int collect(double *sum, int *cnt) {
        int rc = FWI_OK;
        if (hipStreamSynchronize(st) != hipSuccess) rc = FWI_EHIP;
        for (auto &r : recs) {
            float ms = 0.f;
            if (rc == FWI_OK && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
                sum[r.kind] += ms;
                cnt[r.kind] += 1;
            }
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        recs.clear();
        return rc;
    }

    int finish() {
        if (!t) return FWI_OK;
        double sum[K_NKINDS] = {0, 0, 0};
        int cnt[K_NKINDS] = {0, 0, 0};
        const int rc = collect(sum, cnt);
        report(t, launches, updates, sum, cnt);
        return rc;
    }

    static void report(fwi_timing *t, const int *launches, const double *updates,
                       const double *sum, const int *cnt) {
        t->nkinds = K_NKINDS;
        for (int k = 0; k < K_NKINDS; ++k) {
            fwi_kernel_time &o = t->kind[k];
            std::memset(o.name, 0, sizeof(o.name));
            std::strncpy(o.name, kKindName[k], sizeof(o.name) - 1);
            o.launches = launches[k];
            o.timed = cnt[k];
            o.avg_ms = cnt[k] ? sum[k] / cnt[k] : 0.0;
            o.cell_updates = updates[k];
        }
    }
};

// Coefficients, profiles, geometry and the cold arguments.
int setup(const Ptrs &P, const fwi_geom *g, const StreamCold &cold, const float *eps_r,
          const float *sigma, hipStream_t st) {
    const Dims &d = P.L->d;
    int rc = upload_geometry(P, g, cold, st);
    if (rc != FWI_OK) return rc;
    FWI_TRY(launch_coefficients(eps_r, sigma, P.f(P.L->off_Ca), P.f(P.L->off_Cs), d.NX,
                                d.NY, d.pitch, d.dt, st));
    FWI_TRY(launch_profiles(d, P.prof(), st));
    return FWI_OK;
}

// Forward steps [n0, n1) in passes of up to L.depth steps.  E of the pass
// starting at n is read from ein(n); per-level E goes to elev(n) (history /
// segment) or, when elev returns null, the final E of the pass to eout(n).
// The H / CPML state ping-pongs between fwd[cur] and fwd[cur ^ 1].
template <class EIn, class EOut, class ELev>
int forward_passes(const Ptrs &P, FwdStreamArgs a, int n0, int n1, int &cur, EIn ein,
                   EOut eout, ELev elev, bool record, hipStream_t st, Timer &tm) {
    const Layout &L = *P.L;
    State fs[2] = {P.state(L.off_fwd[0], false), P.state(L.off_fwd[1], false)};
    a.record = record ? 1 : 0;
    const double all = (double)L.d.NX * L.d.NY * L.d.S;
    for (int n = n0; n < n1; n += L.depth) {
        a.n = n;
        a.nlev = std::min(L.depth, n1 - n);
        a.E_in = ein(n);
        a.E_lev = elev(n);
        a.E_out = a.E_lev ? nullptr : eout(n);
        a.cur = cur;
        a.Hx_in = fs[cur].Hx;
        a.Hy_in = fs[cur].Hy;
        a.Hx_out = fs[cur ^ 1].Hx;
        a.Hy_out = fs[cur ^ 1].Hy;
        FWI_TRY(tm.run(a.E_lev ? K_FWD_REFWD : K_FWD_SWEEP, all * a.nlev,
                       [&] { return launch_fwd_stream(a, st); }));
        cur ^= 1;
    }
    return FWI_OK;
}

// The forward time loop on a workspace whose coefficients, profiles and
// geometry are in place (record: the traces are written).
int forward_run(const Layout &L, void *ws, bool record, hipStream_t st, Timer &tm) {
    const Dims &d = L.d;
    Ptrs P{static_cast<char *>(ws), &L};
    State fs0 = P.state(L.off_fwd[0], false);
    int rc = zero_state(fs0, d, false, st);
    if (rc != FWI_OK) return rc;
    FWI_TRY(launch_fill(P.slot(0), (size_t)d.S * d.plane, 0.f, st));
    FwdStreamArgs a = fwd_args(P);
    int cur = 0;
    if (L.mode == FWI_SAVE_HISTORY) {
        return forward_passes(
            P, a, 0, d.nt, cur, [&](int n) { return P.slot(n); },
            [&](int) { return (float *)nullptr; }, [&](int n) { return P.slot(n + 1); },
            record, st, tm);
    }
    // E ping-pongs between slots 0 and 1 pass by pass; with checkpoints, the
    // full state (E, H, CPML memories) is copied out every K steps
    const int K = L.ncp > 0 ? L.K : d.nt;
    int e = 0;
    for (int n0 = 0; n0 < d.nt; n0 += K) {
        const int n1 = std::min(d.nt, n0 + K);
        if (L.ncp > 0) {
            const int c = n0 / K;
            char *cp = static_cast<char *>(ws) + L.off_ckpt + (size_t)c * L.ckpt_stride;
            const size_t f = (size_t)d.S * d.plane * sizeof(float);
            FWI_TRY(hipMemcpyAsync(cp, P.slot(e), f, hipMemcpyDeviceToDevice, st));
            State cst = P.state(L.off_ckpt + (size_t)c * L.ckpt_stride + align_up(f), false);
            rc = copy_state(cst, P.state(L.off_fwd[cur], false), d, st);
            if (rc != FWI_OK) return rc;
        }
        rc = forward_passes(
            P, a, n0, n1, cur, [&](int) { return P.slot(e); },
            [&](int) {
                e ^= 1;
                return P.slot(e);
            },
            [&](int) { return (float *)nullptr; }, record, st, tm);
        if (rc != FWI_OK) return rc;
    }
    return FWI_OK;
}

int do_forward(const Layout &L, const fwi_geom *g, const StreamCold &cold,
               const float *eps_r, const float *sigma, void *ws, hipStream_t st,
               Timer &tm) {
    Ptrs P{static_cast<char *>(ws), &L};
    const int rc = setup(P, g, cold, eps_r, sigma, st);
    if (rc != FWI_OK) return rc;
    return forward_run(L, ws, cold.traces != nullptr, st, tm);
}

// The adjoint time loop and imaging; with finalize, the gradients from the
// imaging sums of the layout's shots.
int do_adjoint(const Layout &L, const float *eps_r, const float *sigma, float *g_eps,
               float *g_sig, void *ws, hipStream_t st, Timer &tm, bool finalize = true) {
    const Dims &d = L.d;
    Ptrs P{static_cast<char *>(ws), &L};
    State as[2] = {P.state(L.off_adj[0], true), P.state(L.off_adj[1], true)};
    int rc = zero_state(as[0], d, true, st);
    if (rc != FWI_OK) return rc;
    float *S1 = P.f(L.off_S1), *S2 = P.f(L.off_S2);
    const size_t field = (size_t)d.S * d.plane;
    FWI_TRY(launch_fill(S1, field, 0.f, st));
    FWI_TRY(launch_fill(S2, field, 0.f, st));

    AdjStreamArgs a = adj_args(P);
    int acur = 0;
    const double all = (double)d.NX * d.NY * d.S;
    // adjoint passes over steps [n_lo, n_hi), the forward Ez^{n_lo + k} in slot k.
    // Every pass starts at a multiple of the streaming depth (a partial pass
    // first, at the top), so the grouping of the imaging sums, and with it
    // every rounding, is the same for any checkpoint interval.
    auto adj_range = [&](int n_hi, int n_lo) -> int {
        for (int n_top = n_hi; n_top > n_lo; n_top -= a.nlev) {
            a.nlev = n_top - std::max(n_lo, (n_top - 1) / L.depth * L.depth);
            a.n_top = n_top;
            a.n_base = n_lo;
            a.E_lev = P.slot(0);
            a.cur = acur;
            a.L_in = as[acur].E;
            a.LHx_in = as[acur].Hx;
            a.LHy_in = as[acur].Hy;
            a.L_out = as[acur ^ 1].E;
            a.LHx_out = as[acur ^ 1].Hx;
            a.LHy_out = as[acur ^ 1].Hy;
            FWI_TRY(tm.run(K_ADJ, all * a.nlev, [&] { return launch_adj_stream(a, st); }));
            acur ^= 1;
        }
        return FWI_OK;
    };

    if (L.mode == FWI_SAVE_HISTORY) {
        rc = adj_range(d.nt, 0);
        if (rc != FWI_OK) return rc;
    } else {
        // segment by segment, last first: restore the checkpoint, re-run the
        // segment forward into slots 0..K, then run the adjoint through it
        FwdStreamArgs fa = fwd_args(P);
        const size_t f = field * sizeof(float);
        for (int c = L.ncp - 1; c >= 0; --c) {
            const int n0 = c * L.K, n1 = std::min(d.nt, n0 + L.K);
            const size_t co = L.off_ckpt + (size_t)c * L.ckpt_stride;
            FWI_TRY(hipMemcpyAsync(P.slot(0), P.base + co, f, hipMemcpyDeviceToDevice, st));
            rc = copy_state(P.state(L.off_fwd[0], false), P.state(co + align_up(f), false), d, st);
            if (rc != FWI_OK) return rc;
            int cur = 0;
            rc = forward_passes(
                P, fa, n0, n1, cur, [&](int n) { return P.slot(n - n0); },
                [&](int) { return (float *)nullptr; },
                [&](int n) { return P.slot(n + 1 - n0); }, false, st, tm);
            if (rc != FWI_OK) return rc;
            rc = adj_range(n1, n0);
            if (rc != FWI_OK) return rc;
        }
    }
    if (finalize)
        FWI_TRY(launch_gradient_finalize(eps_r, sigma, S1, S2, d.S, d.plane, g_eps, g_sig,
                                         d.NX, d.NY, d.pitch, d.dt, st));
    return FWI_OK;
}

// fwi_gradient over G >= 2 shot groups, each on a stream of its own (see
// make_group_layout): shot-independent setup and each group's geometry on
// the caller's stream; the groups' forward sweeps; the residual and misfit
// of all shots; the groups' adjoint passes; the gradients from all shots'
// imaging sums in shot order.  The streams join the caller's at each of
// these steps.
int gradient_groups(const Dims &d, int G, const fwi_geom *geom, const float *eps_r,
                    const float *sigma, const float *observed, double *misfit, float *g_eps,
                    float *g_sig, float *traces_out, void *ws, hipStream_t st,
                    fwi_timing *timing) {
    GroupLayout GL;
    int rc = make_group_layout(d, G, GL);
    if (rc != FWI_OK) return rc;
    char *base = static_cast<char *>(ws);
    const Layout &sh = GL.shared;
    Ptrs PS{base, &sh};
    float *traces = traces_out ? traces_out : PS.f(sh.off_trc);
    float *res = PS.f(sh.off_res);
    FWI_TRY(launch_coefficients(eps_r, sigma, PS.f(sh.off_Ca), PS.f(sh.off_Cs), d.NX, d.NY,
                                d.pitch, d.dt, st));
    FWI_TRY(launch_profiles(d, PS.prof(), st));
    fwi_geom gg[kMaxShotGroups];
    for (int g = 0; g < G; ++g) {
        const int s0 = GL.s0[g];
        gg[g] = *geom;
        gg[g].nshots = GL.s0[g + 1] - s0;
        gg[g].src_ij = geom->src_ij + 2 * (size_t)s0;
        gg[g].rec_ij = geom->rec_ij + 2 * (size_t)s0 * d.R;
        gg[g].wavelet = geom->wavelet + (size_t)s0 * d.nt;
        Ptrs P{base, &GL.grp[g]};
        const size_t t0 = (size_t)s0 * d.nt * d.R;
        const StreamCold cold = make_cold(P, &gg[g], traces + t0, res + t0, nullptr);
        rc = upload_geometry(P, &gg[g], cold, st);
        if (rc != FWI_OK) return rc;
    }
    // group 0 runs on the caller's stream, every other group on a stream of
    // its own: G streams in all, which the runtime's default of four
    // hardware queues per process serves side by side up to four groups
    hipStream_t gs[kMaxShotGroups] = {};
    bool made[kMaxShotGroups] = {false, false, false, false};
    hipEvent_t ev[kMaxShotGroups + 1] = {};
    Timer tm[kMaxShotGroups];
    gs[0] = st;
    for (int g = 1; g < G && rc == FWI_OK; ++g) {
        if (hipStreamCreateWithFlags(&gs[g], hipStreamNonBlocking) != hipSuccess)
            rc = FWI_EHIP;
        else
            made[g] = true;
    }
    for (int e = 0; e <= G && rc == FWI_OK; ++e)
        if (hipEventCreateWithFlags(&ev[e], hipEventDisableTiming) != hipSuccess) rc = FWI_EHIP;
    for (int g = 0; g < G; ++g) {
        tm[g].t = timing;
        tm[g].st = gs[g];
    }
    auto fork = [&]() -> int {
        FWI_TRY(hipEventRecord(ev[G], st));
        for (int g = 1; g < G; ++g) FWI_TRY(hipStreamWaitEvent(gs[g], ev[G], 0));
        return FWI_OK;
    };
    // joins every group stream to the caller's, also after a failed step
    auto join = [&]() -> int {
        int r = FWI_OK;
        for (int g = 1; g < G; ++g) {
            if (!made[g] || !ev[g]) continue;
            if (hipEventRecord(ev[g], gs[g]) != hipSuccess ||
                hipStreamWaitEvent(st, ev[g], 0) != hipSuccess)
                r = FWI_EHIP;
        }
        return r;
    };
    // Each group's launches are issued from a host thread of its own, so
    // that every group starts at once: issued from one thread, the last
    // group would wait for the others' thousands of launches to be issued.
    // The threads make the caller's current device theirs before they
    // issue anything.
    int dev = 0;
    if (rc == FWI_OK && hipGetDevice(&dev) != hipSuccess) rc = FWI_EHIP;
    // A group whose thread cannot be started is issued from this thread
    // after the others (no exception leaves the C ABI).
    auto each_group = [&](auto &&phase) -> int {
        int rcs[kMaxShotGroups] = {FWI_OK, FWI_OK, FWI_OK, FWI_OK};
        bool threaded[kMaxShotGroups] = {false, false, false, false};
        std::vector<std::thread> th;
        for (int g = 1; g < G; ++g) {
            try {
                th.emplace_back([&, g] {
                    rcs[g] = hipSetDevice(dev) == hipSuccess ? phase(g) : FWI_EHIP;
                });
                threaded[g] = true;
            } catch (...) {
            }
        }
        rcs[0] = phase(0);
        for (int g = 1; g < G; ++g)
            if (!threaded[g]) rcs[g] = phase(g);
        for (auto &t : th) t.join();
        for (int g = 0; g < G; ++g)
            if (rcs[g] != FWI_OK) return rcs[g];
        return FWI_OK;
    };
    if (rc == FWI_OK) {
        rc = fork();
        if (rc == FWI_OK)
            rc = each_group([&](int g) { return forward_run(GL.grp[g], ws, true, gs[g], tm[g]); });
        const int rj = join();
        if (rc == FWI_OK) rc = rj;
    }
    if (rc == FWI_OK &&
        launch_residual_misfit(traces, observed, res, (size_t)d.S * d.nt * d.R,
                               reinterpret_cast<double *>(base + sh.off_mis), misfit,
                               st) != hipSuccess)
        rc = FWI_EHIP;
    if (rc == FWI_OK) {
        rc = fork();
        if (rc == FWI_OK)
            rc = each_group([&](int g) {
                return do_adjoint(GL.grp[g], eps_r, sigma, nullptr, nullptr, ws, gs[g], tm[g],
                                  false);
            });
        const int rj = join();
        if (rc == FWI_OK) rc = rj;
    }
    if (rc == FWI_OK &&
        launch_gradient_finalize(eps_r, sigma, PS.f(sh.off_S1), PS.f(sh.off_S2), d.S, d.plane,
                                 g_eps, g_sig, d.NX, d.NY, d.pitch, d.dt, st) != hipSuccess)
        rc = FWI_EHIP;
    if (timing) {
        double sum[K_NKINDS] = {0, 0, 0}, upd[K_NKINDS] = {0, 0, 0};
        int cnt[K_NKINDS] = {0, 0, 0}, nl[K_NKINDS] = {0, 0, 0};
        for (int g = 0; g < G; ++g) {
            if (g > 0 && !made[g]) continue;
            const int rt = tm[g].collect(sum, cnt);
            if (rc == FWI_OK) rc = rt;
            for (int k = 0; k < K_NKINDS; ++k) {
                nl[k] += tm[g].launches[k];
                upd[k] += tm[g].updates[k];
            }
        }
        Timer::report(timing, nl, upd, sum, cnt);
        timing->shot_groups = G;
    }
    for (int g = 1; g < G; ++g)
        if (made[g]) {
            if (hipStreamSynchronize(gs[g]) != hipSuccess && rc == FWI_OK) rc = FWI_EHIP;
            (void)hipStreamDestroy(gs[g]);
        }
    for (int e = 0; e <= G; ++e)
        if (ev[e]) (void)hipEventDestroy(ev[e]);
    if (rc != FWI_OK) return rc;
    const size_t cells = (size_t)d.NX * d.NY;
    return check_finite(PS, g_eps, cells, g_sig, cells, misfit, st);
}

int prepare(const fwi_grid *grid, const fwi_geom *geom, int mode, void *ws,
            size_t ws_bytes, Layout &L) {
    Dims d;
    int rc = make_dims(grid, geom, d);
    if (rc != FWI_OK) return rc;
    rc = make_layout(d, mode, L);
    if (rc != FWI_OK) return rc;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0 || ws_bytes < L.total)
        return FWI_ENOMEM;
    return FWI_OK;
}

}  // namespace
}  // namespace fwi

using namespace fwi;
using namespace fwi::host;

extern "C" int fwi_workspace_bytes(const fwi_grid *grid, const fwi_geom *geom,
                                   int save_mode, size_t *bytes) {
    if (!bytes) return FWI_EINVAL;
    Dims d;
    int rc = make_dims(grid, geom, d);
    if (rc != FWI_OK) return rc;
    if (save_mode == -1) return gradient_workspace(d, *bytes);
    Layout L;
    rc = make_layout(d, save_mode, L);
    if (rc != FWI_OK) return rc;
    *bytes = L.total;
    return FWI_OK;
}

extern "C" int fwi_checkpoint_interval(const fwi_grid *grid, const fwi_geom *geom,
                                       int32_t *k) {
    if (!k) return FWI_EINVAL;
    Dims d;
    int rc = make_dims(grid, geom, d);
    if (rc != FWI_OK) return rc;
    *k = choose_k(d, stream_depth(d));
    return FWI_OK;
}

extern "C" int fdtd_forward(const fwi_grid *grid, const fwi_geom *geom,
                            const float *eps_r, const float *sigma, float *traces,
                            int save_mode, void *ws, size_t ws_bytes, void *stream) {
    if (save_mode != FWI_SAVE_NONE && save_mode != FWI_SAVE_CHECKPOINT &&
        save_mode != FWI_SAVE_HISTORY)
        return FWI_EINVAL;
    if (!eps_r || !sigma || !traces) return FWI_EINVAL;
    Layout L;
    int rc = prepare(grid, geom, save_mode, ws, ws_bytes, L);
    if (rc != FWI_OK) return rc;
    Timer tm;
    Ptrs P{static_cast<char *>(ws), &L};
    const StreamCold cold = make_cold(P, geom, traces, nullptr, nullptr);
    hipStream_t st = static_cast<hipStream_t>(stream);
    rc = do_forward(L, geom, cold, eps_r, sigma, ws, st, tm);
    if (rc != FWI_OK) return rc;
    const Dims &d = L.d;
    return check_finite(P, traces, (size_t)d.S * d.nt * d.R, nullptr, 0, nullptr, st);
}

extern "C" int fdtd_adjoint(const fwi_grid *grid, const fwi_geom *geom,
                            const float *eps_r, const float *sigma,
                            const float *residual, float *grad_eps_r,
                            float *grad_sigma, float *src_adjoint, int save_mode,
                            void *ws, size_t ws_bytes, void *stream) {
    if (save_mode != FWI_SAVE_CHECKPOINT && save_mode != FWI_SAVE_HISTORY)
        return FWI_EINVAL;
    if (!eps_r || !sigma || !residual || !grad_eps_r || !grad_sigma) return FWI_EINVAL;
    Layout L;
    int rc = prepare(grid, geom, save_mode, ws, ws_bytes, L);
    if (rc != FWI_OK) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    Ptrs P{static_cast<char *>(ws), &L};
    const StreamCold cold = make_cold(P, geom, nullptr, residual, src_adjoint);
    rc = upload_geometry(P, geom, cold, st);
    if (rc != FWI_OK) return rc;
    Timer tm;
    rc = do_adjoint(L, eps_r, sigma, grad_eps_r, grad_sigma, ws, st, tm);
    if (rc != FWI_OK) return rc;
    const size_t cells = (size_t)L.d.NX * L.d.NY;
    return check_finite(P, grad_eps_r, cells, grad_sigma, cells, nullptr, st);
}

extern "C" int fwi_gradient_ex(const fwi_grid *grid, const fwi_geom *geom, const float *eps_r,
                               const float *sigma, const float *observed, double *misfit,
                               float *grad_eps_r, float *grad_sigma, float *traces_out,
                               void *ws, size_t ws_bytes, void *stream, fwi_timing *timing,
                               int32_t shot_groups) {
    if (!eps_r || !sigma || !observed || !misfit || !grad_eps_r || !grad_sigma)
        return FWI_EINVAL;
    if (timing && timing->sample_every < 1) return FWI_EINVAL;
    if (shot_groups < 0 || shot_groups > kMaxShotGroups) return FWI_EINVAL;
    Dims dd;
    int rc = make_dims(grid, geom, dd);
    if (rc != FWI_OK) return rc;
    const int G = shot_groups ? std::min(shot_groups, dd.S) : auto_shot_groups(dd);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (G > 1) {
        GroupLayout GL;
        rc = make_group_layout(dd, G, GL);
        if (rc != FWI_OK) return rc;
        if (!ws || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0 || ws_bytes < GL.total)
            return FWI_ENOMEM;
        return gradient_groups(dd, G, geom, eps_r, sigma, observed, misfit, grad_eps_r,
                               grad_sigma, traces_out, ws, st, timing);
    }
    Layout L;
    rc = prepare(grid, geom, -1, ws, ws_bytes, L);
    if (rc != FWI_OK) return rc;
    Ptrs P{static_cast<char *>(ws), &L};
    const Dims &d = L.d;
    Timer tm;
    tm.t = timing;
    tm.st = st;
    float *traces = traces_out ? traces_out : P.f(L.off_trc);
    float *res = P.f(L.off_res);
    const StreamCold cold = make_cold(P, geom, traces, res, nullptr);
    rc = do_forward(L, geom, cold, eps_r, sigma, ws, st, tm);
    if (rc == FWI_OK) {
        const size_t ntr = (size_t)d.S * d.nt * d.R;
        if (launch_residual_misfit(traces, observed, res, ntr,
                                   reinterpret_cast<double *>(P.base + L.off_mis), misfit,
                                   st) != hipSuccess)
            rc = FWI_EHIP;
        if (rc == FWI_OK) rc = do_adjoint(L, eps_r, sigma, grad_eps_r, grad_sigma, ws, st, tm);
    }
    const int rc2 = tm.finish();
    if (timing) timing->shot_groups = 1;
    if (rc != FWI_OK) return rc;
    if (rc2 != FWI_OK) return rc2;
    const size_t cells = (size_t)d.NX * d.NY;
    return check_finite(P, grad_eps_r, cells, grad_sigma, cells, misfit, st);
}

extern "C" int fwi_gradient_timed(const fwi_grid *grid, const fwi_geom *geom,
                                  const float *eps_r, const float *sigma,
                                  const float *observed, double *misfit,
                                  float *grad_eps_r, float *grad_sigma,
                                  float *traces_out, void *ws, size_t ws_bytes,
                                  void *stream, fwi_timing *timing) {
    return fwi_gradient_ex(grid, geom, eps_r, sigma, observed, misfit, grad_eps_r, grad_sigma,
                           traces_out, ws, ws_bytes, stream, timing, 0);
}

extern "C" int fwi_gradient(const fwi_grid *grid, const fwi_geom *geom,
                            const float *eps_r, const float *sigma,
                            const float *observed, double *misfit,
                            float *grad_eps_r, float *grad_sigma, float *traces_out,
                            void *ws, size_t ws_bytes, void *stream) {
    return fwi_gradient_ex(grid, geom, eps_r, sigma, observed, misfit, grad_eps_r, grad_sigma,
                           traces_out, ws, ws_bytes, stream, nullptr, 0);
}

extern "C" const char *fwi_strerror(int status) {
    switch (status) {
        case FWI_OK: return "ok";
        case FWI_EINVAL: return "invalid argument (null pointer, size or parameter)";
        case FWI_ECFL: return "time step exceeds the CFL stability bound";
        case FWI_EGEOM: return "source or receiver outside the updated interior";
        case FWI_ENOMEM: return "workspace missing, misaligned or too small";
        case FWI_EHIP: return "HIP runtime or kernel launch failure";
        case FWI_ENONFINITE:
            return "the call completed but its misfit, gradients or traces hold NaN or Inf";
        case FWI_ESCRATCH:
            return "problem needs more scratch than the static array of "
                   "fwi_gradient_static holds (FWI_STATIC_SCRATCH_BYTES)";
        default: return "unknown status";
    }
}
