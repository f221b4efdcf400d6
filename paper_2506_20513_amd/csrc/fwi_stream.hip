// Temporally blocked streaming kernels for the forward step (Algorithm 1)
// and its exact transpose with gradient imaging (Algorithm 2), gfx950.
// Paper: arXiv 2506.20513, Sec. 2.1 Eqs. (3)-(13), Sec. 3.2, Sec. 3.3.
//
// Work decomposition.  One 64-lane wavefront owns one shot, one strip of 64
// consecutive columns and one band of rows.  It marches down the rows of its
// band; at every row it advances K time levels, level l working one row
// behind level l-1 (the forward step needs the row below, the E update the
// row above: the dependency cone widens by one row per level), so each field
// row is read from HBM once per K time steps.  Lane = column; the x
// neighbours of the stencil come from the neighbouring lanes through DPP
// wavefront shifts, so no LDS and no barrier is involved.  The cone also
// widens by one column per level, so after K levels the lanes
// [K, 64-K) of the strip hold valid results: strips overlap by 2K columns and
// only those lanes write.  Rows likewise: a band of rows [y0, y1) starts
// streaming K rows above y0 and stops nlev rows below y1.
//
// Cells outside the grid hold zeros and the PEC ring has Ca = Cs = 0, so the
// same arithmetic is correct everywhere without per-cell predicates (see the
// notes at k_fwd_stream and k_adj_stream).
#include "fwi_internal.h"

#include <type_traits>

namespace fwi {
namespace {

// lane i receives lane i-1's value (lane 0 receives 0)
__device__ __forceinline__ float from_left(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, false));
}
// lane i receives lane i+1's value (lane 63 receives 0)
__device__ __forceinline__ float from_right(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, false));
}

__device__ __forceinline__ int xcol(int i, int NX, int npml) {
    if (i < npml) return i;
    if (i >= NX - 1 - npml) return i - (NX - 1 - npml) + npml;
    return -1;
}
__device__ __forceinline__ int yrow(int j, int NY, int npml) {
    if (j < npml) return j;
    if (j >= NY - 1 - npml) return j - (NY - 1 - npml) + npml;
    return -1;
}

// Blocks are dealt round-robin to the 8 XCDs; renumber them so that each XCD
// works on a contiguous range of the (band, strip, shot) order, with shots
// fastest: the waves co-resident on one XCD then share coefficient rows and
// strip halos through that XCD's L2.
__device__ __forceinline__ int xcd_logical(int b, int nb) {
    const int per = nb / 8, rem = nb % 8;
    const int x = b % 8, k = b / 8;
    return x < rem ? x * (per + 1) + k : rem * (per + 1) + (x - rem) * per + k;
}

__device__ __forceinline__ bool is_lean(const Tiling &t, int strip, int band) {
    return strip >= t.lean_s0 && strip < t.lean_s1 && band >= t.lean_b0 && band < t.lean_b1;
}

// Receivers of shot s on row j whose column lies in [c0, c1): index range
// into the shot's (row, column)-sorted receiver list.
__device__ __forceinline__ void rec_range(const StreamGeom &g, int s, int NY, int R, int j,
                                          int c0, int c1, int &lo, int &hi) {
    const int *rr = g.rrow + (size_t)s * (NY + 1);
    lo = rr[j];
    hi = rr[j + 1];
    if (lo == hi) return;
    const int *rc = g.rcol + (size_t)s * R;
    int a = lo, b = hi;
    while (a < b) {
        const int m = (a + b) >> 1;
        if (rc[m] < c0) a = m + 1; else b = m;
    }
    int e = a, f = hi;
    while (e < f) {
        const int m = (e + f) >> 1;
        if (rc[m] < c1) e = m + 1; else f = m;
    }
    lo = a;
    hi = e;
}

// ---------------------------------------------------------------------------
// Forward: K levels per pass.  Per level and row j (Algorithm 1, stages 1-6):
//   traces  <- Ez^{n+l}(j)                                 (owned cells only)
//   Hx(j)   -= ch/dy * (Ez(j+1)-Ez(j))/kappa_Hy + ch psi_hx'
//   Hy(i)   += ch/dx * (Ez(i+1)-Ez(i))/kappa_Hx + ch psi_hy'
//   Ez      <- Ca Ez + Cs [ dHy/dx/kappa_Ex + psi_ex' - dHx/dy/kappa_Ey - psi_ey' ]
//   Ez(src) -= Cs w[n+l] / (dx dy)                         (every lane holding it)
// With zeros outside the grid, Ez = 0 and Ca = Cs = 0 on the PEC ring, the
// H rows/columns that the oracle does not update (Hx at j = NY-1, Hy at
// i = NX-1) see a zero difference and stay zero, and ring Ez stays zero.
struct FRow {
    float E, Hx, Hy, Ca, Cs, phx, phy, pex, pey;
};

template <int K>
__global__ __launch_bounds__(64) void k_fwd_stream(FwdStreamArgs a) {
    constexpr int OW = 64 - 2 * K;
    const int lane = threadIdx.x;
    const int wid = xcd_logical(blockIdx.x, gridDim.x);
    const int s = wid % a.S;
    const int strip = (wid / a.S) % a.tl.nstrip;
    const int band = wid / (a.S * a.tl.nstrip);
    if (is_lean(a.tl, strip, band)) return;
    const int NX = a.NX, NY = a.NY, P = a.pitch;
    const int x0 = strip * OW;
    const int i = x0 - K + lane;
    const bool inx = i >= 0 && i < NX;
    const bool own = lane >= K && lane < K + OW && inx;
    const int y0 = a.tl.bands[band];
    const int y1 = a.tl.bands[band + 1];
    const int nlev = a.nlev;
    const int cx = inx ? xcol(i, NX, a.npml) : -1;

    const float ch = a.ch, rdx = a.rdx, rdy = a.rdy;
    float chx = 0.f, cxE = 0.f, bHx = 0.f, aHx = 0.f, bEx = 0.f, aEx = 0.f;
    if (inx) {
        chx = ch * rdx * a.p.kHx[i];
        cxE = rdx * a.p.kEx[i];
        bHx = a.p.bHx[i];
        aHx = a.p.aHx[i] * rdx;
        bEx = a.p.bEx[i];
        aEx = a.p.aEx[i] * rdx;
    }
    const int si = a.g.src_ij[2 * s], sj = a.g.src_ij[2 * s + 1];
    const size_t so = (size_t)s * a.plane;
    const float *__restrict__ Ein = a.E_in + so;
    const float *__restrict__ Hxin = a.in.Hx + so;
    const float *__restrict__ Hyin = a.in.Hy + so;
    const float *__restrict__ wav = a.g.wavelet + (size_t)s * a.nt + a.n;
    const int rlast = min(NY - 1, y1 + nlev - 1);   // last input row needed

    auto load = [&](int r) {
        FRow v{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (r >= 0 && r <= rlast && inx) {
            const size_t k = (size_t)r * P + i;
            v.E = Ein[k];
            v.Hx = Hxin[k];
            v.Hy = Hyin[k];
            v.Ca = a.Ca[k];
            v.Cs = a.Cs[k];
            const int ry = yrow(r, NY, a.npml);
            if (ry >= 0) {
                const size_t q = (size_t)s * a.ys + (size_t)ry * P + i;
                v.phx = a.in.phx[q];
                v.pey = a.in.pey[q];
            }
            if (cx >= 0) {
                const size_t q = (size_t)s * a.xs + (size_t)r * a.W + cx;
                v.phy = a.in.phy[q];
                v.pex = a.in.pex[q];
            }
        }
        return v;
    };

    FRow prev[K];
    float hprev[K];
#pragma unroll
    for (int l = 0; l < K; ++l) {
        prev[l] = FRow{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        hprev[l] = 0.f;
    }

    const int T = (y1 - y0) + K + nlev;
    FRow nxt = load(y0 - K);
    for (int t = 0; t < T; ++t) {
        const int r = y0 - K + t;
        FRow in = nxt;
        nxt = load(r + 1);
#pragma unroll
        for (int l = 0; l < K; ++l) {
            if (l < nlev) {
                const int j = r - 1 - l;            // row this level updates
                const FRow &p = prev[l];
                FRow o{0.f, 0.f, 0.f, p.Ca, p.Cs, 0.f, 0.f, 0.f, 0.f};
                const bool jin = j >= 0 && j < NY;
                const bool jown = jin && j >= y0 && j < y1;
                if (a.traces && jown) {             // stage 1: Ez^{n+l} at receivers
                    int lo, hi;
                    rec_range(a.g, s, NY, a.R, j, x0, x0 + OW, lo, hi);
                    for (int q = lo; q < hi; ++q) {
                        if (own && a.g.rcol[(size_t)s * a.R + q] == i)
                            a.traces[((size_t)s * a.nt + a.n + l) * a.R +
                                     a.g.ridx[(size_t)s * a.R + q]] = p.E;
                    }
                }
                if (jin) {
                    const float kHy = a.p.kHy[j], kEy = a.p.kEy[j];
                    const int ry = yrow(j, NY, a.npml);
                    // stages 2-3: H to n+l+1/2
                    const float dEy = in.E - p.E;
                    float hx = p.Hx - (ch * rdy * kHy) * dEy;
                    if (ry >= 0) {
                        o.phx = a.p.bHy[j] * p.phx + (a.p.aHy[j] * rdy) * dEy;
                        hx -= ch * o.phx;
                    }
                    const float dEx = from_right(p.E) - p.E;
                    float hy = p.Hy + chx * dEx;
                    if (cx >= 0) {
                        o.phy = bHx * p.phy + aHx * dEx;
                        hy += ch * o.phy;
                    }
                    // stages 4-6: E to n+l+1
                    const float dHy = hy - from_left(hy);
                    const float dHx = hx - hprev[l];
                    float curl = dHy * cxE - dHx * (rdy * kEy);
                    if (cx >= 0) {
                        o.pex = bEx * p.pex + aEx * dHy;
                        curl += o.pex;
                    }
                    if (ry >= 0) {
                        o.pey = a.p.bEy[j] * p.pey + (a.p.aEy[j] * rdy) * dHx;
                        curl -= o.pey;
                    }
                    float e = p.Ca * p.E + p.Cs * curl;
                    if (j == sj && i == si) e -= p.Cs * wav[l] * a.src_scale;
                    o.E = e;
                    o.Hx = hx;
                    o.Hy = hy;
                }
                hprev[l] = o.Hx;
                if (jown && own) {
                    const size_t k = (size_t)j * P + i;
                    if (a.E_lev) a.E_lev[(size_t)l * a.lev_stride + so + k] = o.E;
                    if (l == nlev - 1) {
                        if (!a.E_lev) a.E_out[so + k] = o.E;
                        a.out.Hx[so + k] = o.Hx;
                        a.out.Hy[so + k] = o.Hy;
                        const int ry = yrow(j, NY, a.npml);
                        if (ry >= 0) {
                            const size_t q = (size_t)s * a.ys + (size_t)ry * P + i;
                            a.out.phx[q] = o.phx;
                            a.out.pey[q] = o.pey;
                        }
                        if (cx >= 0) {
                            const size_t q = (size_t)s * a.xs + (size_t)j * a.W + cx;
                            a.out.phy[q] = o.phy;
                            a.out.pex[q] = o.pex;
                        }
                    }
                }
                prev[l] = in;
                in = o;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Adjoint: K levels per pass, level l taking lambda^{n+1} to lambda^n for
// n = n_top-1-l (the exact transpose of the forward step, followed by the
// adjoint source).  Per row j of a level:
//   on arrival of row j (A1, cell-local):  g = Cs lE,
//       LDx = g/(kx dx) + ax/dx (phi_ex + g),  phi_ex <- bx (phi_ex + g)
//       LDy = -g/(ky dy) + ay/dy (phi_ey - g), phi_ey <- by (phi_ey - g)
//   imaging (A0, owned cells): S1 += lE (E^{n+1} - E^n), S2 += lE (E^{n+1} + E^n)
//   lHy += LDx(i) - LDx(i+1);  lHx += LDy(j) - LDy(j+1)               (A1)
//   h = ch lHy: LDex = (h/kx + ax (phi_hy + h))/dx, phi_hy <- bx (phi_hy + h)
//   h = ch lHx: LDey = (-h/ky + ay (phi_hx - h))/dy, phi_hx <- by (phi_hx - h)
//   lE <- Ca lE + LDex(i-1) - LDex(i) + LDey(j-1) - LDey(j)           (A2)
//   lE(rec) += residual[n]          (A3, every lane holding the receiver)
// With Ca = Cs = 0 on the ring and zeros outside the grid, g, LDx and LDy
// vanish there, so the adjoint H values the oracle never touches stay zero;
// lE on the ring picks up terms but never feeds back (its g is zero), which
// matches the oracle where the ring is not a state variable.
struct ARow {
    float lE, Ca, Cs, ldx, ldy, pex, pey, lHx, lHy, phx, phy, Enp1, s1, s2;
};

template <int K>
__global__ __launch_bounds__(64) void k_adj_stream(AdjStreamArgs a) {
    constexpr int OW = 64 - 2 * K;
    const int lane = threadIdx.x;
    const int wid = xcd_logical(blockIdx.x, gridDim.x);
    const int s = wid % a.S;
    const int strip = (wid / a.S) % a.tl.nstrip;
    const int band = wid / (a.S * a.tl.nstrip);
    if (is_lean(a.tl, strip, band)) return;
    const int NX = a.NX, NY = a.NY, P = a.pitch;
    const int x0 = strip * OW;
    const int i = x0 - K + lane;
    const bool inx = i >= 0 && i < NX;
    const bool own = lane >= K && lane < K + OW && inx;
    const int y0 = a.tl.bands[band];
    const int y1 = a.tl.bands[band + 1];
    const int nlev = a.nlev;
    const int cx = inx ? xcol(i, NX, a.npml) : -1;

    const float ch = a.ch, rdx = a.rdx, rdy = a.rdy;
    float chx = 0.f, cxE = 0.f, bHx = 0.f, aHx = 0.f, bEx = 0.f, aEx = 0.f;
    if (inx) {
        chx = ch * rdx * a.p.kHx[i];
        cxE = rdx * a.p.kEx[i];
        bHx = a.p.bHx[i];
        aHx = a.p.aHx[i] * rdx;
        bEx = a.p.bEx[i];
        aEx = a.p.aEx[i] * rdx;
    }
    const int si = a.src_ij[2 * s], sj = a.src_ij[2 * s + 1];
    const size_t so = (size_t)s * a.plane;
    const float *__restrict__ Lin = a.in.E + so;
    const float *__restrict__ LHxin = a.in.Hx + so;
    const float *__restrict__ LHyin = a.in.Hy + so;
    const int rlast = min(NY - 1, y1 + nlev - 1);

    // A1 for a row on arrival: cell-local terms
    auto arrive = [&](ARow &v, int r) {
        if (r < 0 || r >= NY) return;
        const float g = v.Cs * v.lE;
        const float tx = v.pex + g;
        const float ty = v.pey - g;
        v.ldx = g * cxE + aEx * tx;
        v.ldy = -g * (rdy * a.p.kEy[r]) + (a.p.aEy[r] * rdy) * ty;
        if (cx >= 0) v.pex = bEx * tx;
        if (yrow(r, NY, a.npml) >= 0) v.pey = a.p.bEy[r] * ty;
    };
    auto load = [&](int r) {
        ARow v{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (r >= 0 && r <= rlast && inx) {
            const size_t k = (size_t)r * P + i;
            v.lE = Lin[k];
            v.lHx = LHxin[k];
            v.lHy = LHyin[k];
            v.Ca = a.Ca[k];
            v.Cs = a.Cs[k];
            v.Enp1 = a.E_top[so + k];
            const int ry = yrow(r, NY, a.npml);
            if (ry >= 0) {
                const size_t q = (size_t)s * a.ys + (size_t)ry * P + i;
                v.phx = a.in.phx[q];
                v.pey = a.in.pey[q];
            }
            if (cx >= 0) {
                const size_t q = (size_t)s * a.xs + (size_t)r * a.W + cx;
                v.phy = a.in.phy[q];
                v.pex = a.in.pex[q];
            }
        }
        return v;
    };

    ARow prev[K];
    float ldey_prev[K];
#pragma unroll
    for (int l = 0; l < K; ++l) {
        prev[l] = ARow{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        ldey_prev[l] = 0.f;
    }

    const int T = (y1 - y0) + K + nlev;
    ARow nxt = load(y0 - K);
    for (int t = 0; t < T; ++t) {
        const int r = y0 - K + t;
        ARow in = nxt;
        arrive(in, r);
        nxt = load(r + 1);
#pragma unroll
        for (int l = 0; l < K; ++l) {
            if (l < nlev) {
                const int j = r - 1 - l;
                const int n = a.n_top - 1 - l;
                const ARow &p = prev[l];
                const bool jin = j >= 0 && j < NY;
                const bool jown = jin && j >= y0 && j < y1;
                ARow o{0.f, p.Ca, p.Cs, 0.f, 0.f, p.pex, p.pey, 0.f, 0.f, 0.f, 0.f, 0.f,
                       p.s1, p.s2};
                float ldey = 0.f;
                if (jin) {
                    // forward Ez^n of this row (Ez^{n+1} came with the row)
                    const float en = inx ? a.E_lev[(size_t)(n - a.n_base) * a.lev_stride + so +
                                                   (size_t)j * P + i]
                                         : 0.f;
                    o.Enp1 = en;
                    // A0 imaging with lambda_E^{n+1}
                    if (own && jown) {
                        o.s1 += p.lE * (p.Enp1 - en);
                        o.s2 += p.lE * (p.Enp1 + en);
                    }
                    if (a.src_adjoint && own && j == sj && i == si)
                        a.src_adjoint[(size_t)s * a.nt + n] = -p.Cs * p.lE * a.src_scale;
                    // A1: lambda_H after the transposed E step
                    const float lhy = p.lHy + (p.ldx - from_right(p.ldx));
                    const float lhx = p.lHx + (p.ldy - in.ldy);
                    // A2: transposed H step
                    const float kHy = a.p.kHy[j];
                    const int ry = yrow(j, NY, a.npml);
                    float ldex = lhy * chx;
                    if (cx >= 0) {
                        const float t1 = p.phy + ch * lhy;
                        ldex += aHx * t1;
                        o.phy = bHx * t1;
                    }
                    ldey = -lhx * (ch * rdy * kHy);
                    if (ry >= 0) {
                        const float t2 = p.phx - ch * lhx;
                        ldey += (a.p.aHy[j] * rdy) * t2;
                        o.phx = a.p.bHy[j] * t2;
                    }
                    float le = p.Ca * p.lE + (from_left(ldex) - ldex) + (ldey_prev[l] - ldey);
                    // A3: adjoint source of step n
                    int lo, hi;
                    rec_range(a.g, s, NY, a.R, j, x0 - K, x0 - K + 64, lo, hi);
                    const float *res = a.residual + ((size_t)s * a.nt + n) * a.R;
                    for (int q = lo; q < hi; ++q)
                        if (a.g.rcol[(size_t)s * a.R + q] == i)
                            le += res[a.g.ridx[(size_t)s * a.R + q]];
                    o.lE = le;
                    o.lHx = lhx;
                    o.lHy = lhy;
                }
                ldey_prev[l] = ldey;
                if (jown && own && l == nlev - 1) {
                    const size_t k = (size_t)j * P + i;
                    a.out.E[so + k] = o.lE;
                    a.out.Hx[so + k] = o.lHx;
                    a.out.Hy[so + k] = o.lHy;
                    a.S1[so + k] += o.s1;
                    a.S2[so + k] += o.s2;
                    const int ry = yrow(j, NY, a.npml);
                    if (ry >= 0) {
                        const size_t q = (size_t)s * a.ys + (size_t)ry * P + i;
                        a.out.phx[q] = o.phx;
                        a.out.pey[q] = o.pey;
                    }
                    if (cx >= 0) {
                        const size_t q = (size_t)s * a.xs + (size_t)j * a.W + cx;
                        a.out.phy[q] = o.phy;
                        a.out.pex[q] = o.pex;
                    }
                }
                prev[l] = in;
                in = o;
                arrive(in, j);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Lean kernels: waves of the lean sub-grid (see Tiling), full passes of K
// levels.  No CPML memory (zero away from the strips), kappa = 1, every lane
// inside the grid, so each level is the bare stencil.  A row carries five
// values from level to level; two register sets per level, used alternately
// on even and odd rows, let every level write its output straight into the
// input slot of the next level, so the pipeline needs no register copies.
template <int K>
__global__ __launch_bounds__(64) void k_fwd_lean(FwdStreamArgs a) {
    constexpr int OW = 64 - 2 * K;
    const int lane = threadIdx.x;
    const int nsl = a.tl.lean_s1 - a.tl.lean_s0;
    const int wid = xcd_logical(blockIdx.x, gridDim.x);
    const int s = wid % a.S;
    const int strip = a.tl.lean_s0 + (wid / a.S) % nsl;
    const int band = a.tl.lean_b0 + wid / (a.S * nsl);
    const int P = a.pitch;
    const int x0 = strip * OW;
    const int i = x0 - K + lane;
    const bool own = lane >= K && lane < K + OW;
    const int y0 = a.tl.bands[band], y1 = a.tl.bands[band + 1];
    const float chx = a.ch * a.rdx, chy = a.ch * a.rdy, cxE = a.rdx, cyE = a.rdy;
    const int si = a.g.src_ij[2 * s], sj = a.g.src_ij[2 * s + 1];
    const int rlo = a.g.rspan[2 * s], rhi = a.g.rspan[2 * s + 1];
    const size_t so = (size_t)s * a.plane;
    const float *__restrict__ Ein = a.E_in + so;
    const float *__restrict__ Hxin = a.in.Hx + so;
    const float *__restrict__ Hyin = a.in.Hy + so;
    const float *__restrict__ wav = a.g.wavelet + (size_t)s * a.nt + a.n;
    float *__restrict__ Hxo = a.out.Hx + so;
    float *__restrict__ Hyo = a.out.Hy + so;
    const int rlast = y1 + K - 1;

    float E_[2][K], Hx_[2][K], Hy_[2][K], Ca_[2][K], Cs_[2][K];
#pragma unroll
    for (int l = 0; l < K; ++l) {
        E_[0][l] = E_[1][l] = Hx_[0][l] = Hx_[1][l] = Hy_[0][l] = Hy_[1][l] = 0.f;
        Ca_[0][l] = Ca_[1][l] = Cs_[0][l] = Cs_[1][l] = 0.f;
    }
    float hlast = 0.f;
    float nE = 0.f, nHx = 0.f, nHy = 0.f, nCa = 0.f, nCs = 0.f;
    auto load = [&](int r) {
        if (r <= rlast) {
            const size_t k = (size_t)r * P + i;
            nE = Ein[k];
            nHx = Hxin[k];
            nHy = Hyin[k];
            nCa = a.Ca[k];
            nCs = a.Cs[k];
        } else {
            nE = nHx = nHy = nCa = nCs = 0.f;
        }
    };
    load(y0 - K);

    auto iter = [&](auto pc, int t) {
        constexpr int p = decltype(pc)::value, q = 1 - p;
        const int r = y0 - K + t;
        E_[q][0] = nE; Hx_[q][0] = nHx; Hy_[q][0] = nHy; Ca_[q][0] = nCa; Cs_[q][0] = nCs;
        load(r + 1);
#pragma unroll
        for (int l = 0; l < K; ++l) {
            const int j = r - 1 - l;
            const float pE = E_[p][l], pCa = Ca_[p][l], pCs = Cs_[p][l];
            const float hprev = (l + 1 < K) ? Hx_[p][l + 1] : hlast;
            const bool jown = j >= y0 && j < y1;
            if (a.traces && jown && j >= rlo && j <= rhi) {
                int lo, hi;
                rec_range(a.g, s, a.NY, a.R, j, x0, x0 + OW, lo, hi);
                for (int q2 = lo; q2 < hi; ++q2)
                    if (own && a.g.rcol[(size_t)s * a.R + q2] == i)
                        a.traces[((size_t)s * a.nt + a.n + l) * a.R +
                                 a.g.ridx[(size_t)s * a.R + q2]] = pE;
            }
            const float hx = Hx_[p][l] - chy * (E_[q][l] - pE);
            const float hy = Hy_[p][l] + chx * (from_right(pE) - pE);
            float e = pCa * pE + pCs * ((hy - from_left(hy)) * cxE - (hx - hprev) * cyE);
            if (j == sj && i == si) e -= pCs * wav[l] * a.src_scale;
            if (l + 1 < K) {
                E_[q][l + 1] = e; Hx_[q][l + 1] = hx; Hy_[q][l + 1] = hy;
                Ca_[q][l + 1] = pCa; Cs_[q][l + 1] = pCs;
            } else {
                hlast = hx;
            }
            if (jown && own) {
                const size_t k = (size_t)j * P + i;
                if (a.E_lev) a.E_lev[(size_t)l * a.lev_stride + so + k] = e;
                if (l == K - 1) {
                    if (!a.E_lev) a.E_out[so + k] = e;
                    Hxo[k] = hx;
                    Hyo[k] = hy;
                }
            }
        }
    };
    const int T = (y1 - y0) + 2 * K;
    for (int t = 0; t < T; t += 2) {
        iter(std::integral_constant<int, 0>(), t);
        iter(std::integral_constant<int, 1>(), t + 1);
    }
}

// Lean adjoint.  The imaging sums use a regrouped form of Eqs. (12)-(13):
// because lambda^{nt} = 0 and Ez^0 = 0,
//   S1 = sum_n lambda^{n+1} (E^{n+1} - E^n) = sum_n E^n (lambda^n - lambda^{n+1})
//   S2 = sum_n lambda^{n+1} (E^{n+1} + E^n) = sum_n E^n (lambda^n + lambda^{n+1})
// with lambda^n the state after the adjoint source of step n.  A level then
// needs only the forward Ez^n of its own step; the partial sums of the rows in
// flight live in a small LDS ring, one row per level.
template <int K>
__global__ __launch_bounds__(64) void k_adj_lean(AdjStreamArgs a) {
    static_assert((K & (K - 1)) == 0, "K must be a power of two");
    constexpr int OW = 64 - 2 * K;
    __shared__ float2 ring[K][64];
    const int lane = threadIdx.x;
    const int nsl = a.tl.lean_s1 - a.tl.lean_s0;
    const int wid = xcd_logical(blockIdx.x, gridDim.x);
    const int s = wid % a.S;
    const int strip = a.tl.lean_s0 + (wid / a.S) % nsl;
    const int band = a.tl.lean_b0 + wid / (a.S * nsl);
    const int P = a.pitch, NY = a.NY;
    const int x0 = strip * OW;
    const int i = x0 - K + lane;
    const bool own = lane >= K && lane < K + OW;
    const int y0 = a.tl.bands[band], y1 = a.tl.bands[band + 1];
    const float chx = a.ch * a.rdx, chy = a.ch * a.rdy, cxE = a.rdx, cyE = a.rdy;
    const int si = a.src_ij[2 * s], sj = a.src_ij[2 * s + 1];
    const int rlo = a.g.rspan[2 * s], rhi = a.g.rspan[2 * s + 1];
    const size_t so = (size_t)s * a.plane;
    const float *__restrict__ Lin = a.in.E + so;
    const float *__restrict__ LHxin = a.in.Hx + so;
    const float *__restrict__ LHyin = a.in.Hy + so;
    const float *__restrict__ Ef = a.E_lev + so + i;
    const int rlast = y1 + K - 1;

    float L_[2][K], Ca_[2][K], Cs_[2][K], Hx_[2][K], Hy_[2][K];
    float ldey_prev[K], en_pf[K];
    // forward Ez^{n_l}(j) for level l (n_l = n_top - 1 - l), 0 off the grid
    auto loadE = [&](int l, int j) {
        return (j >= 0 && j < NY)
                   ? Ef[(size_t)(a.n_top - 1 - l - a.n_base) * a.lev_stride + (size_t)j * P]
                   : 0.f;
    };
#pragma unroll
    for (int l = 0; l < K; ++l) {
        L_[0][l] = L_[1][l] = Ca_[0][l] = Ca_[1][l] = Cs_[0][l] = Cs_[1][l] = 0.f;
        Hx_[0][l] = Hx_[1][l] = Hy_[0][l] = Hy_[1][l] = 0.f;
        ldey_prev[l] = 0.f;
        en_pf[l] = loadE(l, y0 - K - 1 - l);
    }
    float nL = 0.f, nCa = 0.f, nCs = 0.f, nHx = 0.f, nHy = 0.f;
    auto load = [&](int r) {
        if (r <= rlast) {
            const size_t k = (size_t)r * P + i;
            nL = Lin[k];
            nHx = LHxin[k];
            nHy = LHyin[k];
            nCa = a.Ca[k];
            nCs = a.Cs[k];
        } else {
            nL = nHx = nHy = nCa = nCs = 0.f;
        }
    };
    load(y0 - K);

    auto iter = [&](auto pc, int t) {
        constexpr int p = decltype(pc)::value, q = 1 - p;
        const int r = y0 - K + t;
        L_[q][0] = nL; Ca_[q][0] = nCa; Cs_[q][0] = nCs; Hx_[q][0] = nHx; Hy_[q][0] = nHy;
        load(r + 1);
#pragma unroll
        for (int l = 0; l < K; ++l) {
            const int j = r - 1 - l;
            const int n = a.n_top - 1 - l;
            const float en = en_pf[l];
            en_pf[l] = loadE(l, j + 1);
            const float pL = L_[p][l], pCa = Ca_[p][l], pCs = Cs_[p][l];
            const bool jown = j >= y0 && j < y1;
            if (a.src_adjoint && own && jown && j == sj && i == si)
                a.src_adjoint[(size_t)s * a.nt + n] = -pCs * pL * a.src_scale;
            // transposed E step, then transposed H step
            const float g = pCs * pL;
            const float ldx = g * cxE;
            const float lhy = Hy_[p][l] + (ldx - from_right(ldx));
            const float lhx = Hx_[p][l] + (Cs_[q][l] * L_[q][l] - g) * cyE;
            const float ldex = lhy * chx;
            const float ldey = -lhx * chy;
            float le = pCa * pL + (from_left(ldex) - ldex) + (ldey_prev[l] - ldey);
            ldey_prev[l] = ldey;
            // adjoint source of step n
            if (j >= rlo && j <= rhi) {
                int lo, hi;
                rec_range(a.g, s, NY, a.R, j, x0 - K, x0 - K + 64, lo, hi);
                const float *res = a.residual + ((size_t)s * a.nt + n) * a.R;
                for (int q2 = lo; q2 < hi; ++q2)
                    if (a.g.rcol[(size_t)s * a.R + q2] == i) le += res[a.g.ridx[(size_t)s * a.R + q2]];
            }
            // imaging
            float2 acc = l == 0 ? make_float2(0.f, 0.f) : ring[j & (K - 1)][lane];
            acc.x += en * (le - pL);
            acc.y += en * (le + pL);
            if (l + 1 < K) {
                ring[j & (K - 1)][lane] = acc;
                L_[q][l + 1] = le; Ca_[q][l + 1] = pCa; Cs_[q][l + 1] = pCs;
                Hx_[q][l + 1] = lhx; Hy_[q][l + 1] = lhy;
            } else if (jown && own) {
                const size_t k = (size_t)j * P + i;
                a.out.E[so + k] = le;
                a.out.Hx[so + k] = lhx;
                a.out.Hy[so + k] = lhy;
                a.S1[so + k] += acc.x;
                a.S2[so + k] += acc.y;
            }
        }
    };
    const int T = (y1 - y0) + 2 * K;
    for (int t = 0; t < T; t += 2) {
        iter(std::integral_constant<int, 0>(), t);
        iter(std::integral_constant<int, 1>(), t + 1);
    }
}

}  // namespace

hipError_t launch_fwd_lean(const FwdStreamArgs &a, hipStream_t st) {
    const unsigned nb = (unsigned)a.S * (a.tl.lean_s1 - a.tl.lean_s0) *
                        (a.tl.lean_b1 - a.tl.lean_b0);
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fwd_lean<kStreamK>, dim3(nb), dim3(64), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_adj_lean(const AdjStreamArgs &a, hipStream_t st) {
    const unsigned nb = (unsigned)a.S * (a.tl.lean_s1 - a.tl.lean_s0) *
                        (a.tl.lean_b1 - a.tl.lean_b0);
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_adj_lean<kStreamK>, dim3(nb), dim3(64), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_fwd_stream(const FwdStreamArgs &a, hipStream_t st) {
    const unsigned nb = (unsigned)a.S * a.tl.nstrip * a.tl.nband;
    hipLaunchKernelGGL(k_fwd_stream<kStreamK>, dim3(nb), dim3(64), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_adj_stream(const AdjStreamArgs &a, hipStream_t st) {
    const unsigned nb = (unsigned)a.S * a.tl.nstrip * a.tl.nband;
    hipLaunchKernelGGL(k_adj_stream<kStreamK>, dim3(nb), dim3(64), 0, st, a);
    return hipGetLastError();
}

}  // namespace fwi
