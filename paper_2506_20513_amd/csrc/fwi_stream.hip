// Temporally blocked streaming kernels for the forward step (Algorithm 1)
// and its exact transpose with gradient imaging (Algorithm 2), gfx950.
// Paper: arXiv 2506.20513, Sec. 2.1 Eqs. (3)-(13), Sec. 3.2, Sec. 3.3.
//
// Work decomposition.  One 64-lane wavefront owns one shot, one strip of 64
// consecutive columns and one band of rows.  It marches down the rows of its
// band; at every row it advances K time levels, level l working one row
// behind level l-1 (the H step needs the row below, the E step the row
// above, so the dependency cone widens by one row per level), so each field
// row is read from HBM once per K time steps.  Lane = column; the x
// neighbours of the stencil come from the neighbouring lanes through DPP
// wavefront shifts, so no barrier is involved.  The cone also widens by one
// column per level: after K levels the lanes [K, 64-K) of the strip hold
// valid results, so strips overlap by 2K columns and only those lanes write.
// Rows likewise: a band [y0, y1) starts streaming K rows above y0 and stops
// nlev rows below y1.
//
// Registers.  A row carries five values from level to level (the three
// fields and the two update coefficients).  Two register sets per level,
// used alternately on even and odd rows, let each level write its output
// straight into the input slot of the next level: the pipeline needs no
// register copies.  The CPML memories are zero away from the CPML strips;
// where they are not, they travel from level to level through a small LDS
// ring (one row slot per level, per wave), level 0 taking them from
// registers.
//
// Cells outside the grid hold zeros and the PEC ring has Ca = Cs = 0, so the
// same arithmetic is correct everywhere without per-cell predicates (see the
// notes at k_fwd and k_adj).
#include "fwi_internal.h"

#include <type_traits>

// Every fused multiply-add below is written out (fmaf), and the compiler may
// not fuse anything else: each cell then sees the same sequence of IEEE
// operations whichever code path (edge or interior strip, quiet or boundary
// row, single or batched problem) computes it, so results do not depend on
// the tiling.  The CPML terms are evaluated only where a CPML coefficient is
// nonzero; elsewhere they would add an exact zero.
#pragma clang fp contract(off)

namespace fwi {
namespace {

// Memory access helpers.  Per-lane accesses go through the global address
// space with a uniform base and a 32-bit offset (SGPR base + VGPR offset
// addressing); read-only tables indexed by uniform values go through the
// constant address space (scalar loads).  Offsets stay below 2^32 bytes by
// the grid-size check on the host.
#define FWI_AS_GLOBAL __attribute__((address_space(1)))
#define FWI_AS_CONST __attribute__((address_space(4)))
template <class T>
__device__ __forceinline__ T ldg(const T *base, unsigned idx) {
    return *(const FWI_AS_GLOBAL T *)((const FWI_AS_GLOBAL char *)base +
                                      (size_t)(idx * (unsigned)sizeof(T)));
}
template <class T>
__device__ __forceinline__ void stg(T *base, unsigned idx, T v) {
    *(FWI_AS_GLOBAL T *)((FWI_AS_GLOBAL char *)base + (size_t)(idx * (unsigned)sizeof(T))) = v;
}
template <class T>
__device__ __forceinline__ T ldc(const T *base, unsigned idx) {
    return ((const FWI_AS_CONST T *)base)[idx];
}
// The per-call cold arguments, read with scalar loads.
using ColdRef = const FWI_AS_CONST StreamCold *;

// The per-level slot pointers of a pass are walked from one base that is
// made opaque at every row iteration: hoisted out of the row loop, eight
// 64-bit pointers per kernel would not fit the scalar registers and would be
// reloaded from spill slots at every use.
template <class T>
__device__ __forceinline__ T *row_base(T *p) {
    asm volatile("" : "+s"(p));
    return p;
}

// lane i receives lane i-1's value (lane 0 receives 0)
__device__ __forceinline__ float from_left(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, false));
}
// lane i receives lane i+1's value (lane 63 receives 0)
__device__ __forceinline__ float from_right(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, false));
}

// Column of the x-direction CPML strip store holding column i, or -1.
__device__ __forceinline__ int xcol(int i, int NX, int npml) {
    if (i < npml) return i;
    if (i >= NX - 1 - npml) return i - (NX - 1 - npml) + npml;
    return -1;
}
// Row of the y-direction CPML strip store holding row j, or -1 (also for
// rows outside the grid).
__device__ __forceinline__ int yrow(int j, int NY, int npml) {
    if (j < 0 || j >= NY) return -1;
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

// Receivers of shot s on row j whose column lies in [c0, c1): index range
// into the shot's (row, column)-sorted receiver list.
__device__ __forceinline__ void rec_range(const int *rrow, const int *rcol, int s, int NY,
                                          int R, int j, int c0, int c1, int &lo, int &hi) {
    const int *rr = rrow + (size_t)s * (NY + 1);
    lo = ldc(rr, j);
    hi = ldc(rr, j + 1);
    if (lo == hi) return;
    const int *rc = rcol + (size_t)s * R;
    int a = lo, b = hi;
    while (a < b) {
        const int m = (a + b) >> 1;
        if (ldc(rc, m) < c0) a = m + 1; else b = m;
    }
    int e = a, f = hi;
    while (e < f) {
        const int m = (e + f) >> 1;
        if (ldc(rc, m) < c1) e = m + 1; else f = m;
    }
    lo = a;
    hi = e;
}

// CPML constants of one row (y direction), scaled by 1/dy where the update
// multiplies by it.  Outside the y strips kappa = 1 and a = 0.
struct RowPml {
    float chy, cyE, bHy, aHy, bEy, aEy;
};
__device__ __forceinline__ RowPml row_pml(ColdRef cold, int j, float ch, float rdy) {
    RowPml r;
    r.chy = ch * rdy * ldc<float>(cold->p.kHy, j);
    r.cyE = rdy * ldc<float>(cold->p.kEy, j);
    r.bHy = ldc<float>(cold->p.bHy, j);
    r.aHy = ldc<float>(cold->p.aHy, j) * rdy;
    r.bEy = ldc<float>(cold->p.bEy, j);
    r.aEy = ldc<float>(cold->p.aEy, j) * rdy;
    return r;
}

// Lane (column) constants: kappa, b and a of the x direction, scaled by 1/dx.
struct ColPml {
    float chx, cxE, bHx, aHx, bEx, aEx;
};
__device__ __forceinline__ ColPml col_pml(ColdRef cold, int i, bool inx, float ch, float rdx) {
    ColPml c{0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (inx) {
        c.chx = ch * rdx * ldg<float>(cold->p.kHx, i);
        c.cxE = rdx * ldg<float>(cold->p.kEx, i);
        c.bHx = ldg<float>(cold->p.bHx, i);
        c.aHx = ldg<float>(cold->p.aHx, i) * rdx;
        c.bEx = ldg<float>(cold->p.bEx, i);
        c.aEx = ldg<float>(cold->p.aEx, i) * rdx;
    }
    return c;
}

// Neighbouring strips of one shot and band handled by one workgroup of the
// single-problem kernels, one wave each (the batched kernels keep one).  The
// two waves of a pair start together on one CU and read each other's halo
// columns; at depth 8 on 2088x1064 x 64 shots this made the gradient 1%
// faster (adjoint 3.50 -> 3.46 ms, re-forward 2.58 -> 2.54 ms per launch),
// at depth 4 on 552x296 x 24 shots 2% slower, so only depth 8 pairs.
template <int K>
struct BlockStrips {
    static constexpr int n = K == kDepthLarge ? 2 : 1;
};

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }
// Index of the calling wave in its workgroup (wave-uniform).
__device__ __forceinline__ int wave_in_block() {
    return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
}

struct WaveTile {
    int s, x0, i, y0, y1;
    bool inx, own, edge, valid;
};
// Workgroup `blk` -> (shot, group of NS neighbouring strips, band); the
// calling wave takes strip NS * group + its index in the workgroup.  An edge
// strip has lanes in a CPML column or outside the grid; interior strips take
// the specialised path (kappa = 1, no CPML memory, no bounds test).
template <int K, int NS = 1>
__device__ __forceinline__ WaveTile wave_tile(const Tiling &tl, int S, int NX, int npml,
                                              int blk) {
    constexpr int OW = 64 - 2 * K;
    WaveTile w;
    const int ngroup = (tl.nstrip + NS - 1) / NS;
    w.s = blk % S;
    const int strip = (blk / S) % ngroup * NS + (NS > 1 ? wave_in_block() : 0);
    const int band = blk / (S * ngroup);
    w.valid = strip < tl.nstrip;
    w.x0 = strip * OW;
    w.i = w.x0 - K + lane_id();
    w.inx = w.i >= 0 && w.i < NX;
    w.own = lane_id() >= K && lane_id() < K + OW && w.inx;
    w.y0 = tl.bands[band];
    w.y1 = tl.bands[band + 1];
    w.edge = !(w.x0 - K >= npml && w.x0 - K + 63 <= NX - 2 - npml);
    return w;
}

// ---------------------------------------------------------------------------
// Forward: K levels per pass (TAIL: nlev < K levels).  Per level and row j
// (Algorithm 1, stages 1-6):
//   traces  <- Ez^{n+l}(j)                                 (owned cells only)
//   Hx(j)   -= ch/dy * (Ez(j+1)-Ez(j))/kappa_Hy + ch psi_hx'
//   Hy(i)   += ch/dx * (Ez(i+1)-Ez(i))/kappa_Hx + ch psi_hy'
//   Ez      <- Ca Ez + Cs [ dHy/dx/kappa_Ex + psi_ex' - dHx/dy/kappa_Ey - psi_ey' ]
//   Ez(src) -= Cs w[n+l] / (dx dy)                         (every lane holding it)
// With zeros outside the grid, Ez = 0 and Ca = Cs = 0 on the PEC ring, the
// H rows/columns that the E update never reads (Hx at j = NY-1, Hy at
// i = NX-1) see a zero difference and stay zero, and ring Ez stays zero.
// psi is a float4 (psi_hx, psi_hy, psi_ex, psi_ey).  LEV: 1 if the pass
// writes every level's Ez (a.E_lev set), 0 if only the final state; fixing
// the choice at compile time keeps the other stores' addresses out of the
// scalar registers.
template <int K, bool EDGE, bool TAIL, int LEV>
__device__ __forceinline__ void fwd_body(const FwdStreamArgs &a, const WaveTile &w,
                                         float4 (*ring)[64]) {
    constexpr int OW = 64 - 2 * K;
    ColdRef cold = (ColdRef)a.cold;
    const int lane = lane_id();
    const int s = w.s, i = w.i, y0 = w.y0, y1 = w.y1;
    const int NY = a.NY, P = a.pitch, npml = a.npml;
    const int nlev = TAIL ? a.nlev : K;
    const bool inx = EDGE ? w.inx : true;
    const bool own = w.own;
    const int cx = EDGE && inx ? xcol(i, a.NX, npml) : -1;
    const bool xp = EDGE && cx >= 0;
    const float ch = a.ch, rdx = a.rdx, rdy = a.rdy;
    ColPml c;
    if (EDGE) {
        c = col_pml(cold, i, inx, ch, rdx);
    } else {
        c = ColPml{ch * rdx, rdx, 0.f, 0.f, 0.f, 0.f};
    }
    const RowPml r0{ch * rdy, rdy, 0.f, 0.f, 0.f, 0.f};
    const int si = ldc<int>(cold->g.src_ij, 2 * s), sj = ldc<int>(cold->g.src_ij, 2 * s + 1);
    const int rlo = ldc<int>(cold->g.rspan, 2 * s), rhi = ldc<int>(cold->g.rspan, 2 * s + 1);
    const size_t so = (size_t)s * a.plane;
    const float *Ein = a.E_in + so;
    const float *Hxin = a.Hx_in + so;
    const float *Hyin = a.Hy_in + so;
    const float *Cap = a.Ca;
    const float *Csp = a.Cs;
    const int rlast = min(NY - 1, y1 + nlev - 1);
    static_assert(LEV == 0 || LEV == 1, "LEV is 0 or 1");
    const bool lev = LEV == 1;
    float *const elev0 = lev ? a.E_lev + so : nullptr;   // level 0 slot of the shot
    const size_t lstr = a.lev_stride;

#pragma unroll
    for (int l = 0; l < K; ++l) ring[l][lane] = make_float4(0.f, 0.f, 0.f, 0.f);

    float E_[2][K], Hx_[2][K], Hy_[2][K], Ca_[2][K], Cs_[2][K];
#pragma unroll
    for (int l = 0; l < K; ++l) {
        E_[0][l] = E_[1][l] = Hx_[0][l] = Hx_[1][l] = Hy_[0][l] = Hy_[1][l] = 0.f;
        Ca_[0][l] = Ca_[1][l] = Cs_[0][l] = Cs_[1][l] = 0.f;
    }
    float4 ps0[2] = {make_float4(0.f, 0.f, 0.f, 0.f), make_float4(0.f, 0.f, 0.f, 0.f)};
    float hlast = 0.f;
    float nE = 0.f, nHx = 0.f, nHy = 0.f, nCa = 0.f, nCs = 0.f;
    float4 nPs = make_float4(0.f, 0.f, 0.f, 0.f);
    auto load = [&](int r) {
        nE = nHx = nHy = nCa = nCs = 0.f;
        nPs = make_float4(0.f, 0.f, 0.f, 0.f);
        if (r >= 0 && r <= rlast && inx) {
            const unsigned k = (unsigned)(r * P + i);
            nE = ldg(Ein, k);
            nHx = ldg(Hxin, k);
            nHy = ldg(Hyin, k);
            nCa = ldg(Cap, k);
            nCs = ldg(Csp, k);
            const int ry = yrow(r, NY, npml);
            if (ry >= 0) {
                const unsigned q = (unsigned)(ry * P + i);
                nPs.x = ldg(cold->fs[a.cur].phx + (size_t)s * a.ys, q);
                nPs.w = ldg(cold->fs[a.cur].pey + (size_t)s * a.ys, q);
            }
            if (xp) {
                const unsigned q = (unsigned)(r * a.W + cx);
                nPs.y = ldg(cold->fs[a.cur].phy + (size_t)s * a.xs, q);
                nPs.z = ldg(cold->fs[a.cur].pex + (size_t)s * a.xs, q);
            }
        }
    };
    load(y0 - K);

    // QUIET: every row of the iteration is owned by the band and lies
    // outside the y-direction CPML, the receiver rows and the source row, so
    // the row-dependent branches are known to be off (same arithmetic).
    auto iter = [&](auto pc, auto quiet, int t) {
        constexpr int p = decltype(pc)::value, q = 1 - p;
        constexpr bool QUIET = decltype(quiet)::value;
        const int r = y0 - K + t;
        E_[q][0] = nE; Hx_[q][0] = nHx; Hy_[q][0] = nHy; Ca_[q][0] = nCa; Cs_[q][0] = nCs;
        ps0[q] = nPs;
        load(r + 1);
        float *el = nullptr;
        if (lev) el = row_base(elev0);
#pragma unroll
        for (int l = 0; l < K; ++l) {
            if (TAIL && l >= nlev) continue;
            const bool last = TAIL ? l == nlev - 1 : l == K - 1;
            const int j = r - 1 - l;
            const float pE = E_[p][l], pCa = Ca_[p][l], pCs = Cs_[p][l];
            const float hprev = (l + 1 < K) ? Hx_[p][l + 1] : hlast;
            const bool jown = QUIET || (j >= y0 && j < y1);
            if (!QUIET && a.record && jown && j >= rlo && j <= rhi) {    // stage 1
                const int *rcol = cold->g.rcol, *ridx = cold->g.ridx;
                int lo, hi;
                rec_range(cold->g.rrow, rcol, s, NY, a.R, j, w.x0, w.x0 + OW, lo, hi);
                float *tr = cold->traces + ((size_t)s * a.nt + a.n + l) * a.R;
                for (int q2 = lo; q2 < hi; ++q2)
                    if (own && ldc(rcol, s * a.R + q2) == i)
                        stg(tr, (unsigned)ldc(ridx, s * a.R + q2), pE);
            }
            const int ry = QUIET ? -1 : yrow(j, NY, npml);
            const bool yp = ry >= 0;
            const RowPml rp = yp ? row_pml(cold, j, ch, rdy) : r0;
            // stages 2-3: H to n+l+1/2
            const float dEy = E_[q][l] - pE;
            const float dEx = from_right(pE) - pE;
            float hx = fmaf(-rp.chy, dEy, Hx_[p][l]);
            float hy = fmaf(c.chx, dEx, Hy_[p][l]);
            float4 ps = make_float4(0.f, 0.f, 0.f, 0.f);
            if (yp || xp) ps = l == 0 ? ps0[p] : ring[j & (K - 1)][lane];
            if (yp) {
                ps.x = fmaf(rp.bHy, ps.x, rp.aHy * dEy);
                hx = fmaf(-ch, ps.x, hx);
            }
            if (xp) {
                ps.y = fmaf(c.bHx, ps.y, c.aHx * dEx);
                hy = fmaf(ch, ps.y, hy);
            }
            // stages 4-6: E to n+l+1
            const float dHy = hy - from_left(hy);
            const float dHx = hx - hprev;
            float curl = fmaf(dHy, c.cxE, -(dHx * rp.cyE));
            if (xp) {
                ps.z = fmaf(c.bEx, ps.z, c.aEx * dHy);
                curl += ps.z;
            }
            if (yp) {
                ps.w = fmaf(rp.bEy, ps.w, rp.aEy * dHx);
                curl -= ps.w;
            }
            float e = fmaf(pCa, pE, pCs * curl);
            if (!QUIET && j == sj && i == si)
                e = fmaf(-(pCs * ldc(cold->g.wavelet + (size_t)s * a.nt, a.n + l)), a.src_scale, e);
            if (l + 1 < K) {
                E_[q][l + 1] = e; Hx_[q][l + 1] = hx; Hy_[q][l + 1] = hy;
                Ca_[q][l + 1] = pCa; Cs_[q][l + 1] = pCs;
                if ((yp || xp) && !last) ring[j & (K - 1)][lane] = ps;
            } else {
                hlast = hx;
            }
            if (jown && own) {
                const unsigned k = (unsigned)(j * P + i);
                if (lev) stg(el, k, e);
                if (last) {
                    if (!lev) stg(a.E_out + so, k, e);
                    stg(a.Hx_out + so, k, hx);
                    stg(a.Hy_out + so, k, hy);
                    if (yp) {
                        const unsigned q2 = (unsigned)(ry * P + i);
                        stg(cold->fs[a.cur ^ 1].phx + (size_t)s * a.ys, q2, ps.x);
                        stg(cold->fs[a.cur ^ 1].pey + (size_t)s * a.ys, q2, ps.w);
                    }
                    if (xp) {
                        const unsigned q2 = (unsigned)(j * a.W + cx);
                        stg(cold->fs[a.cur ^ 1].phy + (size_t)s * a.xs, q2, ps.y);
                        stg(cold->fs[a.cur ^ 1].pex + (size_t)s * a.xs, q2, ps.z);
                    }
                }
            }
            if (lev) el += lstr;
        }
    };
    const int T = (y1 - y0) + K + nlev;
    const int qlo = max(y0, npml), qhi = min(y1, NY - 1 - npml) - 1;   // quiet rows
    // Iterations t and t + 1 touch rows [r - K, r], r = y0 - K + t.  Quiet and
    // other runs of iterations go to separate loops, so the registers of the
    // rare branches are spilled around the quiet loop rather than inside it.
    auto quiet = [&](int t) {
        const int r = y0 - K + t;
        return !TAIL && r - K >= qlo && r <= qhi && (sj < r - K || sj > r) &&
               (!a.record || rhi < r - K || rlo > r);
    };
    int t = 0;
    while (t < T) {
        for (; t < T && !quiet(t); t += 2) {
            iter(std::integral_constant<int, 0>(), std::false_type(), t);
            iter(std::integral_constant<int, 1>(), std::false_type(), t + 1);
        }
        for (; t < T && quiet(t); t += 2) {
            iter(std::integral_constant<int, 0>(), std::true_type(), t);
            iter(std::integral_constant<int, 1>(), std::true_type(), t + 1);
        }
    }
}

template <int K, bool TAIL, int LEV>
__global__ __launch_bounds__(64 * BlockStrips<K>::n) void k_fwd(FwdStreamArgs a) {
    static_assert((K & (K - 1)) == 0, "K must be a power of two");
    constexpr int NS = BlockStrips<K>::n;
    __shared__ float4 ring[NS][K][64];
    const WaveTile w =
        wave_tile<K, NS>(a.tl, a.S, a.NX, a.npml, xcd_logical(blockIdx.x, gridDim.x));
    if (!w.valid) return;
    float4 (*wr)[64] = ring[NS > 1 ? wave_in_block() : 0];
    if (w.edge)
        fwd_body<K, true, TAIL, LEV>(a, w, wr);
    else
        fwd_body<K, false, TAIL, LEV>(a, w, wr);
}

// A struct read from the constant address space dword by dword (scalar
// loads; unused fields are never loaded).
template <class T>
__device__ __forceinline__ T load_const(const T *p, int m) {
    static_assert(sizeof(T) % 4 == 0, "dword-sized struct");
    T v;
    const FWI_AS_CONST unsigned *src = (const FWI_AS_CONST unsigned *)(p + m);
    unsigned *dst = reinterpret_cast<unsigned *>(&v);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(T) / 4); ++k) dst[k] = src[k];
    return v;
}

// The same pass for several independent problems in one launch: problem m
// owns blocks [boff[m], boff[m+1]) of the XCD-renumbered block order and
// reads its arguments from tab[m].
__device__ __forceinline__ int table_entry(const unsigned *boff, int nm, unsigned lb) {
    int lo = 0, hi = nm;                      // boff[lo] <= lb < boff[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (ldc(boff, mid) <= lb) lo = mid; else hi = mid;
    }
    return lo;
}

// LEV as in fwd_body, 0 or 1: the problems of one launch all write every
// level's Ez (segment re-forward) or none does (sweep).  Arguments read from the
// table stay live in registers where kernel arguments would be reloaded, so
// the depth-4 sweep would need 102 VGPRs (4 waves per SIMD); it is held to
// 5 waves, which it reaches without spilling.
template <int K, bool TAIL, int LEV>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(K == kDepthSmall && LEV == 0
                                                                        ? 5
                                                                        : 1))) void
k_fwd_tab(const FwdStreamArgs *tab, const unsigned *boff, int nm) {
    __shared__ float4 ring[K][64];
    const unsigned lb = (unsigned)xcd_logical(blockIdx.x, gridDim.x);
    const int m = table_entry(boff, nm, lb);
    const FwdStreamArgs a = load_const(tab, m);
    const WaveTile w = wave_tile<K>(a.tl, a.S, a.NX, a.npml, (int)(lb - ldc(boff, m)));
    if (w.edge)
        fwd_body<K, true, TAIL, LEV>(a, w, ring);
    else
        fwd_body<K, false, TAIL, LEV>(a, w, ring);
}

// ---------------------------------------------------------------------------
// Adjoint: K levels per pass, level l taking lambda^{n+1} to lambda^n for
// n = n_top-1-l: the exact transpose of the forward step, then the adjoint
// source.  Per row j of a level (row j+1 is the one below):
//   A1  g = Cs lE; LDx = g/(kx dx) + ax/dx (phi_ex + g),  phi_ex <- bx (phi_ex + g)
//                  LDy = -g/(ky dy) + ay/dy (phi_ey - g), phi_ey <- by (phi_ey - g)
//       lHy += LDx(i) - LDx(i+1);  lHx += LDy(j) - LDy(j+1)
//   A2  h = ch lHy: LDex = (h/kx + ax (phi_hy + h))/dx, phi_hy <- bx (phi_hy + h)
//       h = ch lHx: LDey = (-h/ky + ay (phi_hx - h))/dy, phi_hx <- by (phi_hx - h)
//       lE <- Ca lE + LDex(i-1) - LDex(i) + LDey(j-1) - LDey(j)
//   A3  lE(rec) += residual[n]                     (every lane holding it)
// With Ca = Cs = 0 on the ring and zeros outside the grid, g and hence the
// adjoint H values the forward never reads stay zero; lE on the ring picks
// up terms but never feeds back (its g is zero), matching the oracle where
// the ring is not a state variable.  phi is a float4 (phi_ex, phi_ey,
// phi_hx, phi_hy).
//
// Imaging uses a regrouped form of Eqs. (12)-(13): because lambda^{nt} = 0
// and Ez^0 = 0,
//   S1 = sum_n lambda^{n+1} (E^{n+1} - E^n) = sum_n E^n (lambda^n - lambda^{n+1})
//   S2 = sum_n lambda^{n+1} (E^{n+1} + E^n) = sum_n E^n (lambda^n + lambda^{n+1})
// with lambda^n the state after the adjoint source of step n, so a level
// needs only the forward Ez^n of its own step (prefetched a row ahead); the
// partial sums of the rows in flight live in a second LDS ring.
template <int K, bool EDGE, bool TAIL>
__device__ __forceinline__ void adj_body(const AdjStreamArgs &a, const WaveTile &w,
                                         float4 (*ring)[64], float2 (*img)[64]) {
    ColdRef cold = (ColdRef)a.cold;
    const int lane = lane_id();
    const int s = w.s, i = w.i, y0 = w.y0, y1 = w.y1;
    const int NY = a.NY, P = a.pitch, npml = a.npml;
    const int nlev = TAIL ? a.nlev : K;
    const bool inx = EDGE ? w.inx : true;
    const bool own = w.own;
    const int cx = EDGE && inx ? xcol(i, a.NX, npml) : -1;
    const bool xp = EDGE && cx >= 0;
    const float ch = a.ch, rdx = a.rdx, rdy = a.rdy;
    ColPml c;
    if (EDGE) {
        c = col_pml(cold, i, inx, ch, rdx);
    } else {
        c = ColPml{ch * rdx, rdx, 0.f, 0.f, 0.f, 0.f};
    }
    const RowPml r0{ch * rdy, rdy, 0.f, 0.f, 0.f, 0.f};
    const int si = ldc<int>(cold->g.src_ij, 2 * s), sj = ldc<int>(cold->g.src_ij, 2 * s + 1);
    const int rlo = ldc<int>(cold->g.rspan, 2 * s), rhi = ldc<int>(cold->g.rspan, 2 * s + 1);
    const size_t so = (size_t)s * a.plane;
    const float *Lin = a.L_in + so;
    const float *LHxin = a.LHx_in + so;
    const float *LHyin = a.LHy_in + so;
    const float *Cap = a.Ca;
    const float *Csp = a.Cs;
    const int rlast = min(NY - 1, y1 + nlev - 1);

    // forward Ez^{n_l}(j) of level l (n_l = n_top - 1 - l) from its slot el;
    // level l's slot is lstr floats below level l-1's.  Only the imaging sums
    // use it, and only the cells the wave owns (its band's rows, its owned
    // columns) store those, so other cells skip the load and take 0: their
    // values are another wave's to image.
    auto loadE = [&](const float *el, int j) {
        return (j >= y0 && j < y1 && own) ? ldg(el, (unsigned)(j * P + i)) : 0.f;
    };
    const float *const etop = a.E_lev + (size_t)(a.n_top - 1 - a.n_base) * a.lev_stride + so;
    const size_t lstr = a.lev_stride;

    float L_[2][K], Ca_[2][K], Cs_[2][K], Hx_[2][K], Hy_[2][K];
    float ldey_prev[K], en_pf[K];
#pragma unroll
    for (int l = 0; l < K; ++l) {
        ring[l][lane] = make_float4(0.f, 0.f, 0.f, 0.f);
        L_[0][l] = L_[1][l] = Ca_[0][l] = Ca_[1][l] = Cs_[0][l] = Cs_[1][l] = 0.f;
        Hx_[0][l] = Hx_[1][l] = Hy_[0][l] = Hy_[1][l] = 0.f;
        ldey_prev[l] = 0.f;
        en_pf[l] = (TAIL && l >= nlev) ? 0.f : loadE(etop - (size_t)l * lstr, y0 - K - 1 - l);
    }
    float4 ph0[2] = {make_float4(0.f, 0.f, 0.f, 0.f), make_float4(0.f, 0.f, 0.f, 0.f)};
    float nL = 0.f, nCa = 0.f, nCs = 0.f, nHx = 0.f, nHy = 0.f;
    float4 nPh = make_float4(0.f, 0.f, 0.f, 0.f);
    auto load = [&](int r) {
        nL = nCa = nCs = nHx = nHy = 0.f;
        nPh = make_float4(0.f, 0.f, 0.f, 0.f);
        if (r >= 0 && r <= rlast && inx) {
            const unsigned k = (unsigned)(r * P + i);
            nL = ldg(Lin, k);
            nHx = ldg(LHxin, k);
            nHy = ldg(LHyin, k);
            nCa = ldg(Cap, k);
            nCs = ldg(Csp, k);
            const int ry = yrow(r, NY, npml);
            if (ry >= 0) {
                const unsigned q = (unsigned)(ry * P + i);
                nPh.y = ldg(cold->as[a.cur].pey + (size_t)s * a.ys, q);
                nPh.z = ldg(cold->as[a.cur].phx + (size_t)s * a.ys, q);
            }
            if (xp) {
                const unsigned q = (unsigned)(r * a.W + cx);
                nPh.x = ldg(cold->as[a.cur].pex + (size_t)s * a.xs, q);
                nPh.w = ldg(cold->as[a.cur].phy + (size_t)s * a.xs, q);
            }
        }
    };
    load(y0 - K);

    // QUIET: as in the forward pass (rows j and j + 1 of every level clear of
    // the y-direction CPML, the receiver rows and the source row).
    auto iter = [&](auto pc, auto quiet, int t) {
        constexpr int p = decltype(pc)::value, q = 1 - p;
        constexpr bool QUIET = decltype(quiet)::value;
        const int r = y0 - K + t;
        L_[q][0] = nL; Ca_[q][0] = nCa; Cs_[q][0] = nCs; Hx_[q][0] = nHx; Hy_[q][0] = nHy;
        ph0[q] = nPh;
        load(r + 1);
        const float *el = row_base(etop);
#pragma unroll
        for (int l = 0; l < K; ++l) {
            if (TAIL && l >= nlev) continue;
            const bool last = TAIL ? l == nlev - 1 : l == K - 1;
            const int j = r - 1 - l;
            const int n = a.n_top - 1 - l;
            const float en = en_pf[l];
            en_pf[l] = loadE(el, j + 1);
            el -= lstr;
            const float pL = L_[p][l], pCa = Ca_[p][l], pCs = Cs_[p][l];
            const bool jown = QUIET || (j >= y0 && j < y1);
            if (!QUIET && jown && j == sj && cold->src_adjoint && own && i == si)
                stg(cold->src_adjoint + (size_t)s * a.nt, (unsigned)n, -pCs * pL * a.src_scale);
            const int ry = QUIET ? -1 : yrow(j, NY, npml);
            const int ry1 = QUIET ? -1 : yrow(j + 1, NY, npml);
            const bool yp = ry >= 0, yp1 = ry1 >= 0;
            const RowPml rp = yp ? row_pml(cold, j, ch, rdy) : r0;
            const RowPml rp1 = yp1 ? row_pml(cold, j + 1, ch, rdy) : r0;
            float4 ph = make_float4(0.f, 0.f, 0.f, 0.f);
            if (yp || xp) ph = l == 0 ? ph0[p] : ring[j & (K - 1)][lane];
            // A1: transposed E step, row j and the LDy of row j+1
            const float g = pCs * pL;
            float ldx = g * c.cxE;
            float ldy = -g * rp.cyE;
            if (xp) {
                const float tx = ph.x + g;
                ldx = fmaf(c.aEx, tx, ldx);
                ph.x = c.bEx * tx;
            }
            if (yp) {
                const float ty = ph.y - g;
                ldy = fmaf(rp.aEy, ty, ldy);
                ph.y = rp.bEy * ty;
            }
            const float gn = Cs_[q][l] * L_[q][l];
            float ldyn = -gn * rp1.cyE;
            if (yp1) {
                const float pey1 = l == 0 ? ph0[q].y : ring[(j + 1) & (K - 1)][lane].y;
                ldyn = fmaf(rp1.aEy, pey1 - gn, ldyn);
            }
            const float lhy = Hy_[p][l] + (ldx - from_right(ldx));
            const float lhx = Hx_[p][l] + (ldy - ldyn);
            // A2: transposed H step
            float ldex = lhy * c.chx;
            if (xp) {
                const float t1 = fmaf(ch, lhy, ph.w);
                ldex = fmaf(c.aHx, t1, ldex);
                ph.w = c.bHx * t1;
            }
            float ldey = -lhx * rp.chy;
            if (yp) {
                const float t2 = fmaf(-ch, lhx, ph.z);
                ldey = fmaf(rp.aHy, t2, ldey);
                ph.z = rp.bHy * t2;
            }
            float le = fmaf(pCa, pL, from_left(ldex) - ldex) + (ldey_prev[l] - ldey);
            ldey_prev[l] = ldey;
            // A3: adjoint source of step n
            if (!QUIET && j >= rlo && j <= rhi) {
                const int *rcol = cold->g.rcol, *ridx = cold->g.ridx;
                int lo, hi;
                rec_range(cold->g.rrow, rcol, s, NY, a.R, j, w.x0 - K, w.x0 - K + 64, lo, hi);
                const float *res = cold->residual + ((size_t)s * a.nt + n) * a.R;
                for (int q2 = lo; q2 < hi; ++q2)
                    if (ldc(rcol, s * a.R + q2) == i) le += ldc(res, ldc(ridx, s * a.R + q2));
            }
            // imaging
            float2 acc = l == 0 ? make_float2(0.f, 0.f) : img[j & (K - 1)][lane];
            acc.x = fmaf(en, le - pL, acc.x);
            acc.y = fmaf(en, le + pL, acc.y);
            if (l + 1 < K) {
                L_[q][l + 1] = le; Ca_[q][l + 1] = pCa; Cs_[q][l + 1] = pCs;
                Hx_[q][l + 1] = lhx; Hy_[q][l + 1] = lhy;
                if (!last) {
                    img[j & (K - 1)][lane] = acc;
                    if (yp || xp) ring[j & (K - 1)][lane] = ph;
                }
            }
            if (last && jown && own) {
                const unsigned k = (unsigned)(j * P + i);
                stg(a.L_out + so, k, le);
                stg(a.LHx_out + so, k, lhx);
                stg(a.LHy_out + so, k, lhy);
                stg(a.S1 + so, k, ldg(a.S1 + so, k) + acc.x);
                stg(a.S2 + so, k, ldg(a.S2 + so, k) + acc.y);
                if (yp) {
                    const unsigned q2 = (unsigned)(ry * P + i);
                    stg(cold->as[a.cur ^ 1].pey + (size_t)s * a.ys, q2, ph.y);
                    stg(cold->as[a.cur ^ 1].phx + (size_t)s * a.ys, q2, ph.z);
                }
                if (xp) {
                    const unsigned q2 = (unsigned)(j * a.W + cx);
                    stg(cold->as[a.cur ^ 1].pex + (size_t)s * a.xs, q2, ph.x);
                    stg(cold->as[a.cur ^ 1].phy + (size_t)s * a.xs, q2, ph.w);
                }
            }
        }
    };
    const int T = (y1 - y0) + K + nlev;
    const int qlo = max(y0, npml), qhi = min(y1, NY - 1 - npml) - 2;   // rows j, j + 1 quiet
    // Iterations t and t + 1 touch rows [r - K, r], r = y0 - K + t.  Quiet and
    // other runs of iterations go to separate loops, so the registers of the
    // rare branches are spilled around the quiet loop rather than inside it.
    auto quiet = [&](int t) {
        const int r = y0 - K + t;
        return !TAIL && r - K >= qlo && r <= qhi && (sj < r - K || sj > r) &&
               (rhi < r - K || rlo > r);
    };
    int t = 0;
    while (t < T) {
        for (; t < T && !quiet(t); t += 2) {
            iter(std::integral_constant<int, 0>(), std::false_type(), t);
            iter(std::integral_constant<int, 1>(), std::false_type(), t + 1);
        }
        for (; t < T && quiet(t); t += 2) {
            iter(std::integral_constant<int, 0>(), std::true_type(), t);
            iter(std::integral_constant<int, 1>(), std::true_type(), t + 1);
        }
    }
}

template <int K, bool TAIL>
__global__ __launch_bounds__(64 * BlockStrips<K>::n) void k_adj(AdjStreamArgs a) {
    static_assert((K & (K - 1)) == 0, "K must be a power of two");
    constexpr int NS = BlockStrips<K>::n;
    __shared__ float4 ring[NS][K][64];
    __shared__ float2 img[NS][K][64];
    const WaveTile w =
        wave_tile<K, NS>(a.tl, a.S, a.NX, a.npml, xcd_logical(blockIdx.x, gridDim.x));
    if (!w.valid) return;
    const int wb = NS > 1 ? wave_in_block() : 0;
    if (w.edge)
        adj_body<K, true, TAIL>(a, w, ring[wb], img[wb]);
    else
        adj_body<K, false, TAIL>(a, w, ring[wb], img[wb]);
}

template <int K, bool TAIL>
__global__ __launch_bounds__(64) void k_adj_tab(const AdjStreamArgs *tab, const unsigned *boff,
                                                int nm) {
    __shared__ float4 ring[K][64];
    __shared__ float2 img[K][64];
    const unsigned lb = (unsigned)xcd_logical(blockIdx.x, gridDim.x);
    const int m = table_entry(boff, nm, lb);
    const AdjStreamArgs a = load_const(tab, m);
    const WaveTile w = wave_tile<K>(a.tl, a.S, a.NX, a.npml, (int)(lb - ldc(boff, m)));
    if (w.edge)
        adj_body<K, true, TAIL>(a, w, ring, img);
    else
        adj_body<K, false, TAIL>(a, w, ring, img);
}

}  // namespace

unsigned stream_blocks(int S, const Tiling &tl) {
    return (unsigned)S * tl.nstrip * tl.nband;
}

template <int K, int LEV>
void launch_fwd_table_lev(const FwdStreamArgs *tab, const unsigned *boff, int nm,
                          unsigned nblocks, bool tail, hipStream_t st) {
    if (tail)
        hipLaunchKernelGGL((k_fwd_tab<K, true, LEV>), dim3(nblocks), dim3(64), 0, st, tab, boff,
                           nm);
    else
        hipLaunchKernelGGL((k_fwd_tab<K, false, LEV>), dim3(nblocks), dim3(64), 0, st, tab, boff,
                           nm);
}

template <int K>
hipError_t launch_fwd_table_depth(const FwdStreamArgs *tab, const unsigned *boff, int nm,
                                  unsigned nblocks, bool tail, int lev, hipStream_t st) {
    if (lev == 0)
        launch_fwd_table_lev<K, 0>(tab, boff, nm, nblocks, tail, st);
    else
        launch_fwd_table_lev<K, 1>(tab, boff, nm, nblocks, tail, st);
    return hipGetLastError();
}

template <int K>
hipError_t launch_adj_table_depth(const AdjStreamArgs *tab, const unsigned *boff, int nm,
                                  unsigned nblocks, bool tail, hipStream_t st) {
    if (tail)
        hipLaunchKernelGGL((k_adj_tab<K, true>), dim3(nblocks), dim3(64), 0, st, tab, boff, nm);
    else
        hipLaunchKernelGGL((k_adj_tab<K, false>), dim3(nblocks), dim3(64), 0, st, tab, boff, nm);
    return hipGetLastError();
}

hipError_t launch_fwd_table(const FwdStreamArgs *tab, const unsigned *boff, int nm,
                            unsigned nblocks, int depth, bool tail, int lev, hipStream_t st) {
    if (lev != 0 && lev != 1) return hipErrorInvalidValue;
    if (nblocks == 0) return hipSuccess;
    if (depth == kDepthSmall)
        return launch_fwd_table_depth<kDepthSmall>(tab, boff, nm, nblocks, tail, lev, st);
    if (depth == kDepthLarge)
        return launch_fwd_table_depth<kDepthLarge>(tab, boff, nm, nblocks, tail, lev, st);
    return hipErrorInvalidValue;
}

hipError_t launch_adj_table(const AdjStreamArgs *tab, const unsigned *boff, int nm,
                            unsigned nblocks, int depth, bool tail, hipStream_t st) {
    if (nblocks == 0) return hipSuccess;
    if (depth == kDepthSmall)
        return launch_adj_table_depth<kDepthSmall>(tab, boff, nm, nblocks, tail, st);
    if (depth == kDepthLarge)
        return launch_adj_table_depth<kDepthLarge>(tab, boff, nm, nblocks, tail, st);
    return hipErrorInvalidValue;
}

// Workgroups of a single-problem pass at depth K: BlockStrips<K>::n
// neighbouring strips each.
template <int K>
unsigned single_blocks(int S, const Tiling &tl) {
    constexpr int NS = BlockStrips<K>::n;
    return (unsigned)S * ((tl.nstrip + NS - 1) / NS) * tl.nband;
}

// Single-problem passes at the problem's temporal depth (a.tl.depth);
// nlev < depth takes the partial-pass variant.
template <int K>
hipError_t launch_fwd_depth(const FwdStreamArgs &a, hipStream_t st) {
    const unsigned nb = single_blocks<K>(a.S, a.tl);
    const bool full = a.nlev == K;
    if (a.E_lev) {
        if (full)
            hipLaunchKernelGGL((k_fwd<K, false, 1>), dim3(nb), dim3(64 * BlockStrips<K>::n), 0, st, a);
        else
            hipLaunchKernelGGL((k_fwd<K, true, 1>), dim3(nb), dim3(64 * BlockStrips<K>::n), 0, st, a);
    } else {
        if (full)
            hipLaunchKernelGGL((k_fwd<K, false, 0>), dim3(nb), dim3(64 * BlockStrips<K>::n), 0, st, a);
        else
            hipLaunchKernelGGL((k_fwd<K, true, 0>), dim3(nb), dim3(64 * BlockStrips<K>::n), 0, st, a);
    }
    return hipGetLastError();
}

template <int K>
hipError_t launch_adj_depth(const AdjStreamArgs &a, hipStream_t st) {
    const unsigned nb = single_blocks<K>(a.S, a.tl);
    if (a.nlev == K)
        hipLaunchKernelGGL((k_adj<K, false>), dim3(nb), dim3(64 * BlockStrips<K>::n), 0, st, a);
    else
        hipLaunchKernelGGL((k_adj<K, true>), dim3(nb), dim3(64 * BlockStrips<K>::n), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_fwd_stream(const FwdStreamArgs &a, hipStream_t st) {
    if (a.nlev < 1 || a.nlev > a.tl.depth) return hipErrorInvalidValue;
    if (a.tl.depth == kDepthLarge) return launch_fwd_depth<kDepthLarge>(a, st);
    if (a.tl.depth == kDepthSmall) return launch_fwd_depth<kDepthSmall>(a, st);
    return hipErrorInvalidValue;
}

hipError_t launch_adj_stream(const AdjStreamArgs &a, hipStream_t st) {
    if (a.nlev < 1 || a.nlev > a.tl.depth) return hipErrorInvalidValue;
    if (a.tl.depth == kDepthLarge) return launch_adj_depth<kDepthLarge>(a, st);
    if (a.tl.depth == kDepthSmall) return launch_adj_depth<kDepthSmall>(a, st);
    return hipErrorInvalidValue;
}

}  // namespace fwi
