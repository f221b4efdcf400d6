// HIP kernels for gfx950: coefficients, CPML profiles, the fused forward
// step (H half step + H-CPML + E step + E-CPML + source + receivers), the
// fused adjoint step (imaging + transposed E step + transposed H step), the
// adjoint-source injection, gradient scaling and the misfit reduction.
//
// Paper: arXiv 2506.20513, Sec. 2.1 (Eqs. (3)-(13)), Sec. 3.2 (kernels),
// Sec. 3.3 (Algorithms 1 and 2).
//
// Layout: every field of every shot is a [NY][pitch] plane (x contiguous,
// pitch = NX rounded up to 64 floats), shots stacked [S][NY][pitch].  One
// thread owns one cell (i, j) and loops over the shots, so per-cell model
// coefficients and CPML profiles are read once per step for all shots and
// the imaging correlation is summed over shots in registers in shot order.
#include "fwi_internal.h"

#include <math.h>

namespace fwi {
namespace {

constexpr int kBX = 64;   // one wave64 spans 64 consecutive cells of a row
constexpr int kBY = 4;

// Column of the x-direction CPML strip store that holds cell column i, or -1.
__device__ __forceinline__ int xcol(int i, int NX, int npml) {
    if (i < npml) return i;
    if (i >= NX - 1 - npml) return i - (NX - 1 - npml) + npml;
    return -1;
}
// Row of the y-direction CPML strip store that holds cell row j, or -1.
__device__ __forceinline__ int yrow(int j, int NY, int npml) {
    if (j < npml) return j;
    if (j >= NY - 1 - npml) return j - (NY - 1 - npml) + npml;
    return -1;
}
__device__ __forceinline__ bool ecell(int i, int j, int NX, int NY) {
    return i >= 1 && i <= NX - 2 && j >= 1 && j <= NY - 2;
}

// ---------------------------------------------------------------------------
// Update coefficients, double precision, stored as float (Sec. 3.2,
// coefficient kernel): Ca = EB/EA, Cs = 1/EA; sigma > 100 S/m => 0.
__global__ void k_coefficients(const float *__restrict__ eps_r,
                               const float *__restrict__ sigma,
                               float *__restrict__ Ca, float *__restrict__ Cs,
                               int NX, int NY, int pitch, double dt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= NX || j >= NY) return;
    const double er = eps_r[(size_t)j * NX + i];
    const double sg = sigma[(size_t)j * NX + i];
    float ca = 0.f, cs = 0.f;
    if (!(sg > kPecSigma)) {
        const double EA = kEps0 * er / dt + 0.5 * sg;
        const double EB = kEps0 * er / dt - 0.5 * sg;
        ca = (float)(EB / EA);
        cs = (float)(1.0 / EA);
    }
    Ca[(size_t)j * pitch + i] = ca;
    Cs[(size_t)j * pitch + i] = cs;
}

// CPML grading along one axis of n cells (convolutional PML, polynomial
// order m); rho is the normalised depth into the layer from the interior.
__device__ double pml_rho(int n, int npml, double pos) {
    if (npml <= 0) return 0.0;
    const double lo = (double)npml, hi = (double)(n - 1 - npml);
    if (pos < lo) return (lo - pos) / npml;
    if (pos > hi) return (pos - hi) / npml;
    return 0.0;
}

__device__ void pml_coeffs(double rho, double d, double dt, int m, double scale,
                           double kmax, double amax, float *b, float *a,
                           float *ki) {
    const double eta0 = sqrt(kMu0 / kEps0);
    const double smax = scale * 0.8 * (m + 1) / (eta0 * d);
    const double rm = pow(rho, (double)m);
    const double sp = smax * rm;
    const double kap = 1.0 + (kmax - 1.0) * rm;
    const double al = amax * (1.0 - rho);
    const double bb = exp(-(sp / kap + al) * dt / kEps0);
    const double aa = sp > 0.0 ? sp * (bb - 1.0) / (kap * (sp + kap * al)) : 0.0;
    *b = (float)bb;
    *a = (float)aa;
    *ki = (float)(1.0 / kap);
}

__global__ void k_profiles(Dims d, Profiles p) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < d.NX) {
        pml_coeffs(pml_rho(d.NX, d.npml, t), d.dx, d.dt, d.cpml_order,
                   d.cpml_sigma_scale, d.cpml_kappa_max, d.cpml_alpha_max,
                   &p.bEx[t], &p.aEx[t], &p.kEx[t]);
        pml_coeffs(pml_rho(d.NX, d.npml, t + 0.5), d.dx, d.dt, d.cpml_order,
                   d.cpml_sigma_scale, d.cpml_kappa_max, d.cpml_alpha_max,
                   &p.bHx[t], &p.aHx[t], &p.kHx[t]);
    } else if (t < d.NX + d.NY) {
        const int u = t - d.NX;
        pml_coeffs(pml_rho(d.NY, d.npml, u), d.dy, d.dt, d.cpml_order,
                   d.cpml_sigma_scale, d.cpml_kappa_max, d.cpml_alpha_max,
                   &p.bEy[u], &p.aEy[u], &p.kEy[u]);
        pml_coeffs(pml_rho(d.NY, d.npml, u + 0.5), d.dy, d.dt, d.cpml_order,
                   d.cpml_sigma_scale, d.cpml_kappa_max, d.cpml_alpha_max,
                   &p.bHy[u], &p.aHy[u], &p.kHy[u]);
    }
}

__global__ void k_fill(float *__restrict__ dst, size_t n, float v) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride)
        dst[t] = v;
}

// ---------------------------------------------------------------------------
// Forward step n for all shots (Algorithm 1, stages 1-6):
//   1. traces[s][n][r] = Ez^n(rec)                      (reads E_in only)
//   2-3. Hx, Hy to n+1/2 with H-CPML memories           (Eqs. (4), (5))
//   4-5. Ez to n+1 with E-CPML memories                 (Eq. (3), Sec. 3.2)
//   6. Ez(src) -= Cs w[n] / (dx dy)
// Reads state `in` / E_in, writes `out` / E_out (ping-pong), so the H values
// at (i-1, j) and (i, j-1) that the E update needs are recomputed from the
// unmodified inputs instead of being exchanged.
__global__ __launch_bounds__(kBX * kBY) void k_fwd_step(FwdStepArgs a) {
    if (a.g.traces) {
        const int nthr = gridDim.x * gridDim.y * (kBX * kBY);
        const int tid = (blockIdx.y * gridDim.x + blockIdx.x) * (kBX * kBY) +
                        threadIdx.y * kBX + threadIdx.x;
        const int tot = a.S * a.R;
        for (int t = tid; t < tot; t += nthr) {
            const int s = t / a.R, r = t - s * a.R;
            const int ri = a.g.rec_ij[2 * t], rj = a.g.rec_ij[2 * t + 1];
            a.g.traces[((size_t)s * a.nt + a.n) * a.R + r] =
                a.E_in[(size_t)s * a.plane + (size_t)rj * a.pitch + ri];
        }
    }
    const int i = blockIdx.x * kBX + threadIdx.x;
    const int j = blockIdx.y * kBY + threadIdx.y;
    const int NX = a.NX, NY = a.NY, npml = a.npml;
    if (i >= NX || j >= NY) return;

    const size_t k = (size_t)j * a.pitch + i;
    const bool hx_c = j <= NY - 2;
    const bool hy_c = i <= NX - 2;
    const bool e_c = ecell(i, j, NX, NY);
    const int cx = xcol(i, NX, npml), ry = yrow(j, NY, npml);
    const int cxm = e_c ? xcol(i - 1, NX, npml) : -1;
    const int rym = e_c ? yrow(j - 1, NY, npml) : -1;

    const float kHy0 = a.p.kHy[j], bHy0 = a.p.bHy[j], aHy0 = a.p.aHy[j];
    const float kHx0 = a.p.kHx[i], bHx0 = a.p.bHx[i], aHx0 = a.p.aHx[i];
    float kHxm = 0.f, bHxm = 0.f, aHxm = 0.f, kHym = 0.f, bHym = 0.f, aHym = 0.f;
    float kEx0 = 0.f, bEx0 = 0.f, aEx0 = 0.f, kEy0 = 0.f, bEy0 = 0.f, aEy0 = 0.f;
    float Ca = 0.f, Cs = 0.f;
    if (e_c) {
        kHxm = a.p.kHx[i - 1]; bHxm = a.p.bHx[i - 1]; aHxm = a.p.aHx[i - 1];
        kHym = a.p.kHy[j - 1]; bHym = a.p.bHy[j - 1]; aHym = a.p.aHy[j - 1];
        kEx0 = a.p.kEx[i]; bEx0 = a.p.bEx[i]; aEx0 = a.p.aEx[i];
        kEy0 = a.p.kEy[j]; bEy0 = a.p.bEy[j]; aEy0 = a.p.aEy[j];
        Ca = a.Ca[k];
        Cs = a.Cs[k];
    }
    const float rdx = a.rdx, rdy = a.rdy, ch = a.ch;

    for (int s = 0; s < a.S; ++s) {
        const size_t so = (size_t)s * a.plane;
        const float *__restrict__ E = a.E_in + so;
        const float e0 = E[k];
        float hxn = 0.f, hyn = 0.f;
        if (hx_c) {
            const float de = (E[k + a.pitch] - e0) * rdy;
            float ps = 0.f;
            if (ry >= 0) {
                const size_t q = (size_t)s * a.ys + (size_t)ry * a.pitch + i;
                ps = bHy0 * a.in.phx[q] + aHy0 * de;
                a.out.phx[q] = ps;
            }
            hxn = a.in.Hx[so + k] - ch * (de * kHy0 + ps);
            a.out.Hx[so + k] = hxn;
        }
        if (hy_c) {
            const float de = (E[k + 1] - e0) * rdx;
            float ps = 0.f;
            if (cx >= 0) {
                const size_t q = (size_t)s * a.xs + (size_t)j * a.W + cx;
                ps = bHx0 * a.in.phy[q] + aHx0 * de;
                a.out.phy[q] = ps;
            }
            hyn = a.in.Hy[so + k] + ch * (de * kHx0 + ps);
            a.out.Hy[so + k] = hyn;
        }
        float en = 0.f;
        if (e_c) {
            // Hy^{n+1/2}(i-1, j) and Hx^{n+1/2}(i, j-1), recomputed
            float de = (e0 - E[k - 1]) * rdx;
            float ps = 0.f;
            if (cxm >= 0)
                ps = bHxm * a.in.phy[(size_t)s * a.xs + (size_t)j * a.W + cxm] + aHxm * de;
            const float hym = a.in.Hy[so + k - 1] + ch * (de * kHxm + ps);
            de = (e0 - E[k - a.pitch]) * rdy;
            ps = 0.f;
            if (rym >= 0)
                ps = bHym * a.in.phx[(size_t)s * a.ys + (size_t)rym * a.pitch + i] + aHym * de;
            const float hxm = a.in.Hx[so + k - a.pitch] - ch * (de * kHym + ps);

            const float Dx = (hyn - hym) * rdx;
            const float Dy = (hxn - hxm) * rdy;
            float px = 0.f, py = 0.f;
            if (cx >= 0) {
                const size_t q = (size_t)s * a.xs + (size_t)j * a.W + cx;
                px = bEx0 * a.in.pex[q] + aEx0 * Dx;
                a.out.pex[q] = px;
            }
            if (ry >= 0) {
                const size_t q = (size_t)s * a.ys + (size_t)ry * a.pitch + i;
                py = bEy0 * a.in.pey[q] + aEy0 * Dy;
                a.out.pey[q] = py;
            }
            en = Ca * e0 + Cs * ((Dx * kEx0 + px) - (Dy * kEy0 + py));
            if (i == a.g.src_ij[2 * s] && j == a.g.src_ij[2 * s + 1])
                en -= Cs * a.g.wavelet[(size_t)s * a.nt + a.n] * a.src_scale;
        }
        a.E_out[so + k] = en;
    }
}

// ---------------------------------------------------------------------------
// Adjoint step n for all shots: the exact transpose of k_fwd_step (stages
// 2-6), preceded by the imaging condition (Algorithm 2, stage 6; Eqs. (12),
// (13)).  in = lambda^{n+1}, out = lambda^n before the adjoint source of
// step n (k_adj_inject).  Gather form: each thread recomputes the adjoint
// difference terms of its four neighbours instead of scattering.
//   A0  S1 += lE (E^{n+1} - E^n), S2 += lE (E^{n+1} + E^n)   (summed over s)
//   A1  g = Cs lE; LDx = g/kx + ax (phi_ex + g); LDy = -g/ky + ay (phi_ey - g)
//       phi_e* <- b*(...); lHy += (LDx(i) - LDx(i+1))/dx;
//       lHx += (LDy(j) - LDy(j+1))/dy; lE <- Ca lE
//   A2  h = ch lH; LDex = h/kx + ax (phi_hy + h); LDey = -h/ky + ay (phi_hx - h)
//       phi_h* <- b*(...); lE += (LDex(i-1) - LDex(i))/dx + (LDey(j-1) - LDey(j))/dy
__global__ __launch_bounds__(kBX * kBY) void k_adj_step(AdjStepArgs a) {
    const int i = blockIdx.x * kBX + threadIdx.x;
    const int j = blockIdx.y * kBY + threadIdx.y;
    const int NX = a.NX, NY = a.NY, npml = a.npml;
    if (i >= NX || j >= NY) return;

    const size_t k = (size_t)j * a.pitch + i;
    const int P = a.pitch;
    const bool e0c = ecell(i, j, NX, NY);
    const bool exm = ecell(i - 1, j, NX, NY), exp_ = ecell(i + 1, j, NX, NY);
    const bool eym = ecell(i, j - 1, NX, NY), eyp = ecell(i, j + 1, NX, NY);
    const bool hx_c = j <= NY - 2, hy_c = i <= NX - 2;
    const int cx0 = xcol(i, NX, npml), ry0 = yrow(j, NY, npml);
    const int cxm = i >= 1 ? xcol(i - 1, NX, npml) : -1;
    const int cxp = i + 1 < NX ? xcol(i + 1, NX, npml) : -1;
    const int rym = j >= 1 ? yrow(j - 1, NY, npml) : -1;
    const int ryp = j + 1 < NY ? yrow(j + 1, NY, npml) : -1;

    const float Ca0 = e0c ? a.Ca[k] : 0.f, Cs0 = e0c ? a.Cs[k] : 0.f;
    const float Csxm = exm ? a.Cs[k - 1] : 0.f, Csxp = exp_ ? a.Cs[k + 1] : 0.f;
    const float Csym = eym ? a.Cs[k - P] : 0.f, Csyp = eyp ? a.Cs[k + P] : 0.f;
    const Profiles &p = a.p;
    const float kEx0 = p.kEx[i], aEx0 = p.aEx[i], bEx0 = p.bEx[i];
    const float kEy0 = p.kEy[j], aEy0 = p.aEy[j], bEy0 = p.bEy[j];
    const float kExm = exm ? p.kEx[i - 1] : 0.f, aExm = exm ? p.aEx[i - 1] : 0.f;
    const float kExp = exp_ ? p.kEx[i + 1] : 0.f, aExp = exp_ ? p.aEx[i + 1] : 0.f;
    const float kEym = eym ? p.kEy[j - 1] : 0.f, aEym = eym ? p.aEy[j - 1] : 0.f;
    const float kEyp = eyp ? p.kEy[j + 1] : 0.f, aEyp = eyp ? p.aEy[j + 1] : 0.f;
    const float kHx0 = p.kHx[i], aHx0 = p.aHx[i], bHx0 = p.bHx[i];
    const float kHy0 = p.kHy[j], aHy0 = p.aHy[j], bHy0 = p.bHy[j];
    const float kHxm = e0c ? p.kHx[i - 1] : 0.f, aHxm = e0c ? p.aHx[i - 1] : 0.f;
    const float kHym = e0c ? p.kHy[j - 1] : 0.f, aHym = e0c ? p.aHy[j - 1] : 0.f;
    const float rdx = a.rdx, rdy = a.rdy, ch = a.ch;

    float acc1 = 0.f, acc2 = 0.f;
    for (int s = 0; s < a.S; ++s) {
        const size_t so = (size_t)s * a.plane;
        const size_t xo = (size_t)s * a.xs + (size_t)j * a.W;
        const size_t yo = (size_t)s * a.ys;
        const float *__restrict__ L = a.in.E + so;
        const float l0 = L[k];
        const float lxm = exm ? L[k - 1] : 0.f, lxp = exp_ ? L[k + 1] : 0.f;
        const float lym = eym ? L[k - P] : 0.f, lyp = eyp ? L[k + P] : 0.f;

        // A0: imaging with lambda_E^{n+1}
        if (e0c) {
            const float e1 = a.E_np1[so + k], e = a.E_n[so + k];
            acc1 += l0 * (e1 - e);
            acc2 += l0 * (e1 + e);
            if (a.src_adjoint && i == a.src_ij[2 * s] && j == a.src_ij[2 * s + 1])
                a.src_adjoint[(size_t)s * a.nt + a.n] = -Cs0 * l0 * a.src_scale;
        }

        // A1: adjoints of the E-step differences at (i-1..i+1, j), (i, j-1..j+1)
        float ldx0 = 0.f, ldxm = 0.f, ldxp = 0.f, ldy0 = 0.f, ldym = 0.f, ldyp = 0.f;
        if (e0c) {
            const float g = Cs0 * l0;
            const float tx = g + (cx0 >= 0 ? a.in.pex[xo + cx0] : 0.f);
            ldx0 = g * kEx0 + aEx0 * tx;
            if (cx0 >= 0) a.out.pex[xo + cx0] = bEx0 * tx;
            const float ty = (ry0 >= 0 ? a.in.pey[yo + (size_t)ry0 * P + i] : 0.f) - g;
            ldy0 = -g * kEy0 + aEy0 * ty;
            if (ry0 >= 0) a.out.pey[yo + (size_t)ry0 * P + i] = bEy0 * ty;
        }
        if (exm) {
            const float g = Csxm * lxm;
            ldxm = g * kExm + aExm * (g + (cxm >= 0 ? a.in.pex[xo + cxm] : 0.f));
        }
        if (exp_) {
            const float g = Csxp * lxp;
            ldxp = g * kExp + aExp * (g + (cxp >= 0 ? a.in.pex[xo + cxp] : 0.f));
        }
        if (eym) {
            const float g = Csym * lym;
            ldym = -g * kEym + aEym * ((rym >= 0 ? a.in.pey[yo + (size_t)rym * P + i] : 0.f) - g);
        }
        if (eyp) {
            const float g = Csyp * lyp;
            ldyp = -g * kEyp + aEyp * ((ryp >= 0 ? a.in.pey[yo + (size_t)ryp * P + i] : 0.f) - g);
        }
        const float lhy0 = hy_c ? a.in.Hy[so + k] + (ldx0 - ldxp) * rdx : 0.f;
        const float lhx0 = hx_c ? a.in.Hx[so + k] + (ldy0 - ldyp) * rdy : 0.f;

        // A2: adjoints of the H-step differences at (i, j), (i-1, j), (i, j-1)
        float lex0 = 0.f, ley0 = 0.f, lexm = 0.f, leym = 0.f;
        if (hy_c) {
            const float h = ch * lhy0;
            const float t = (cx0 >= 0 ? a.in.phy[xo + cx0] : 0.f) + h;
            lex0 = h * kHx0 + aHx0 * t;
            if (cx0 >= 0) a.out.phy[xo + cx0] = bHx0 * t;
        }
        if (hx_c) {
            const float h = ch * lhx0;
            const float t = (ry0 >= 0 ? a.in.phx[yo + (size_t)ry0 * P + i] : 0.f) - h;
            ley0 = -h * kHy0 + aHy0 * t;
            if (ry0 >= 0) a.out.phx[yo + (size_t)ry0 * P + i] = bHy0 * t;
        }
        float le = 0.f;
        if (e0c) {
            const float lhym = a.in.Hy[so + k - 1] + (ldxm - ldx0) * rdx;
            float h = ch * lhym;
            float t = (cxm >= 0 ? a.in.phy[xo + cxm] : 0.f) + h;
            lexm = h * kHxm + aHxm * t;
            const float lhxm = a.in.Hx[so + k - P] + (ldym - ldy0) * rdy;
            h = ch * lhxm;
            t = (rym >= 0 ? a.in.phx[yo + (size_t)rym * P + i] : 0.f) - h;
            leym = -h * kHym + aHym * t;
            le = Ca0 * l0 + (lexm - lex0) * rdx + (leym - ley0) * rdy;
        }
        a.out.E[so + k] = le;
        a.out.Hx[so + k] = lhx0;
        a.out.Hy[so + k] = lhy0;
    }
    if (e0c) {
        a.S1[k] += acc1;
        a.S2[k] += acc2;
    }
}

// Adjoint source of step n (Algorithm 2, stage 1): lE(rec) += residual[n].
// Receivers of a shot that share a cell were grouped on the host (order =
// receivers sorted by cell, glen = group length at the group's first entry,
// 0 elsewhere), so each cell is written by exactly one thread and the sum
// order is fixed.
__global__ void k_adj_inject(const float *__restrict__ res, float *__restrict__ lE,
                             const int *__restrict__ rec_ij,
                             const int *__restrict__ order,
                             const int *__restrict__ glen, int S, int R, int nt,
                             int n, size_t plane, int pitch) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= S * R) return;
    const int len = glen[t];
    if (len == 0) return;
    const int s = t / R;
    const float *rr = res + ((size_t)s * nt + n) * R;
    const int *ord = order + t;
    float sum = 0.f;
    for (int q = 0; q < len; ++q) sum += rr[ord[q]];
    const int r0 = ord[0];
    const int ri = rec_ij[2 * ((size_t)s * R + r0)], rj = rec_ij[2 * ((size_t)s * R + r0) + 1];
    lE[(size_t)s * plane + (size_t)rj * pitch + ri] += sum;
}

// g_eps = -eps0/(dt EA) S1, g_sig = -S2/(2 EA) on updated, non-PEC cells.
__global__ void k_gradient_finalize(const float *__restrict__ eps_r,
                                    const float *__restrict__ sigma,
                                    const float *__restrict__ S1,
                                    const float *__restrict__ S2,
                                    float *__restrict__ ge, float *__restrict__ gs,
                                    int NX, int NY, int pitch, double dt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= NX || j >= NY) return;
    const size_t o = (size_t)j * NX + i;
    float a = 0.f, b = 0.f;
    const double sg = sigma[o];
    if (ecell(i, j, NX, NY) && !(sg > kPecSigma)) {
        const double EA = kEps0 * (double)eps_r[o] / dt + 0.5 * sg;
        a = (float)(-kEps0 / (dt * EA) * (double)S1[(size_t)j * pitch + i]);
        b = (float)(-(double)S2[(size_t)j * pitch + i] / (2.0 * EA));
    }
    ge[o] = a;
    gs[o] = b;
}

// residual = traces - observed; per-block partial sums of r^2 in double.
__global__ __launch_bounds__(256) void k_residual(const float *__restrict__ tr,
                                                  const float *__restrict__ ob,
                                                  float *__restrict__ res, size_t n,
                                                  double *__restrict__ partials) {
    __shared__ double red[256];
    double acc = 0.0;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
        const float r = tr[t] - ob[t];
        res[t] = r;
        acc += (double)r * (double)r;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_misfit_final(const double *__restrict__ partials,
                                                      int np, double *__restrict__ misfit) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int t = threadIdx.x; t < np; t += 256) acc += partials[t];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *misfit = 0.5 * red[0];
}

dim3 cell_grid(int NX, int NY) {
    return dim3((NX + kBX - 1) / kBX, (NY + kBY - 1) / kBY);
}

}  // namespace

hipError_t launch_coefficients(const float *eps_r, const float *sigma, float *Ca,
                               float *Cs, int NX, int NY, int pitch, double dt,
                               hipStream_t st) {
    hipLaunchKernelGGL(k_coefficients, dim3((NX + 255) / 256, NY), dim3(256), 0, st,
                       eps_r, sigma, Ca, Cs, NX, NY, pitch, dt);
    return hipGetLastError();
}

hipError_t launch_profiles(const Dims &d, const Profiles &p, hipStream_t st) {
    const int n = d.NX + d.NY;
    hipLaunchKernelGGL(k_profiles, dim3((n + 255) / 256), dim3(256), 0, st, d, p);
    return hipGetLastError();
}

hipError_t launch_fill(float *dst, size_t n, float v, hipStream_t st) {
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, st, dst, n, v);
    return hipGetLastError();
}

hipError_t launch_fwd_step(const FwdStepArgs &a, hipStream_t st) {
    hipLaunchKernelGGL(k_fwd_step, cell_grid(a.NX, a.NY), dim3(kBX, kBY), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_adj_step(const AdjStepArgs &a, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_step, cell_grid(a.NX, a.NY), dim3(kBX, kBY), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_adj_inject(const float *residual, float *lE, const int *rec_ij,
                             const int *order, const int *glen, int S, int R,
                             int nt, int n, size_t plane, int pitch,
                             hipStream_t st) {
    const int tot = S * R;
    hipLaunchKernelGGL(k_adj_inject, dim3((tot + 255) / 256), dim3(256), 0, st,
                       residual, lE, rec_ij, order, glen, S, R, nt, n, plane, pitch);
    return hipGetLastError();
}

hipError_t launch_gradient_finalize(const float *eps_r, const float *sigma,
                                    const float *S1, const float *S2,
                                    float *g_eps, float *g_sig, int NX, int NY,
                                    int pitch, double dt, hipStream_t st) {
    hipLaunchKernelGGL(k_gradient_finalize, dim3((NX + 255) / 256, NY), dim3(256), 0,
                       st, eps_r, sigma, S1, S2, g_eps, g_sig, NX, NY, pitch, dt);
    return hipGetLastError();
}

hipError_t launch_residual_misfit(const float *traces, const float *observed,
                                  float *residual, size_t n, double *partials,
                                  double *misfit, hipStream_t st) {
    hipLaunchKernelGGL(k_residual, dim3(kMisfitBlocks), dim3(256), 0, st, traces,
                       observed, residual, n, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_misfit_final, dim3(1), dim3(256), 0, st, partials,
                       kMisfitBlocks, misfit);
    return hipGetLastError();
}

}  // namespace fwi
