/*
 * FP64 CPU oracle for 2D TM-mode FDTD in lossy media with CPML, its exact
 * discrete adjoint, and the zero-lag cross-correlation gradients with
 * respect to relative permittivity and conductivity.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code, header or constant with the
 * HIP library: every constant and formula is written out again here.
 *
 * Paper: "Fast ground penetrating radar dual-parameter full waveform
 * inversion method accelerated by hybrid compilation of CUDA kernel
 * function and PyTorch" (arXiv 2506.20513).
 *
 * Plain loops over the whole grid, full-size CPML auxiliary arrays (zero
 * where the profile vanishes), double precision throughout.  OpenMP only
 * splits independent rows; every cell is computed by the same formula in
 * the same order as a serial run, so results are thread-count independent.
 *
 * Grid convention: total grid NX x NY cells, x fastest (index i), y = depth
 * (index j).  Arrays are [NY][NX].  The interior of nx x ny cells is padded
 * by npml CPML cells on each side.  Ez lives on integer nodes (i, j), Hx on
 * (i, j+1/2), Hy on (i+1/2, j).  The outer ring of Ez is a PEC wall held at 0.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Free-space constants (Sec. 2.1: mu is the free-space permeability). */
static const double ORC_PI = 3.14159265358979323846;
#define ORC_C0 299792458.0
#define ORC_MU0 (4.0e-7 * ORC_PI)
#define ORC_EPS0 (1.0 / (ORC_MU0 * ORC_C0 * ORC_C0))

/* Conductivity above which a cell is treated as a perfect conductor and gets
 * zero update coefficients (Sec. 3.2, coefficient kernel). */
#define ORC_PEC_SIGMA 100.0

double orc_eps0(void) { return ORC_EPS0; }
double orc_mu0(void) { return ORC_MU0; }
double orc_c0(void) { return ORC_C0; }

/* ------------------------------------------------------------------------ */
/* CPML profiles along one axis.                                             */
/*                                                                           */
/* The paper names a PML but does not give its formulation (Sec. 3.2, "two  */
/* for updating the PML boundaries"; Tables 2-4, pmlthick).  Reading used:  */
/* the convolutional PML of Roden & Gedney (2000) with a polynomial grading */
/* of order m.  Normalised depth rho in [0,1] measured from the interior    */
/* edge; E nodes at integer positions, H nodes at +1/2.                      */
/*   sigma_p = sigma_max rho^m, sigma_max = scale 0.8 (m+1) / (eta0 d)       */
/*   kappa   = 1 + (kappa_max - 1) rho^m                                     */
/*   alpha   = alpha_max (1 - rho)                                           */
/*   b = exp(-(sigma_p/kappa + alpha) dt / eps0)                             */
/*   a = sigma_p (b - 1) / (kappa (sigma_p + kappa alpha))   (0 if sigma_p=0) */
/* Outputs: b, a and 1/kappa at E positions (bE, aE, kiE) and H positions.   */
/* ------------------------------------------------------------------------ */
static double orc_rho(int n, int npml, double pos)
{
    /* pos is the node position in cell units on an axis of n cells */
    if (npml <= 0) return 0.0;
    double lo = (double)npml;            /* first interior E node */
    double hi = (double)(n - 1 - npml);  /* last interior E node */
    if (pos < lo) return (lo - pos) / (double)npml;
    if (pos > hi) return (pos - hi) / (double)npml;
    return 0.0;
}

static void orc_one_profile(double rho, double d, double dt, int order,
                            double sigma_scale, double kappa_max,
                            double alpha_max, double *b, double *a,
                            double *kinv)
{
    double eta0 = sqrt(ORC_MU0 / ORC_EPS0);
    double sigma_max = sigma_scale * 0.8 * (order + 1) / (eta0 * d);
    double rm = pow(rho, (double)order);
    double sp = sigma_max * rm;
    double kappa = 1.0 + (kappa_max - 1.0) * rm;
    double alpha = alpha_max * (1.0 - rho);
    double bb = exp(-(sp / kappa + alpha) * dt / ORC_EPS0);
    double aa = 0.0;
    if (sp > 0.0) aa = sp * (bb - 1.0) / (kappa * (sp + kappa * alpha));
    *b = bb;
    *a = aa;
    *kinv = 1.0 / kappa;
}

void orc_cpml_profile(int n, int npml, double d, double dt, int order,
                      double sigma_scale, double kappa_max, double alpha_max,
                      double *bE, double *aE, double *kiE, double *bH,
                      double *aH, double *kiH)
{
    for (int i = 0; i < n; ++i) {
        orc_one_profile(orc_rho(n, npml, (double)i), d, dt, order, sigma_scale,
                        kappa_max, alpha_max, &bE[i], &aE[i], &kiE[i]);
        orc_one_profile(orc_rho(n, npml, (double)i + 0.5), d, dt, order,
                        sigma_scale, kappa_max, alpha_max, &bH[i], &aH[i],
                        &kiH[i]);
    }
}

/* ------------------------------------------------------------------------ */
/* Update coefficients (Sec. 3.2, coefficient kernel; semi-implicit form):   */
/*   EA = eps0 eps_r / dt + sigma / 2,  EB = eps0 eps_r / dt - sigma / 2     */
/*   Ca = EB / EA (self-update),  Cs = 1 / EA (curl and source scale)        */
/*   sigma > 100 S/m: Ca = Cs = 0 (perfect conductor).                       */
/* ------------------------------------------------------------------------ */
void orc_coefficients(int ncell, const double *eps_r, const double *sigma,
                      double dt, double *Ca, double *Cs)
{
    for (int k = 0; k < ncell; ++k) {
        if (sigma[k] > ORC_PEC_SIGMA) {
            Ca[k] = 0.0;
            Cs[k] = 0.0;
        } else {
            double EA = ORC_EPS0 * eps_r[k] / dt + 0.5 * sigma[k];
            double EB = ORC_EPS0 * eps_r[k] / dt - 0.5 * sigma[k];
            Ca[k] = EB / EA;
            Cs[k] = 1.0 / EA;
        }
    }
}

/* A problem description shared by the forward and adjoint sweeps. */
typedef struct {
    int NX, NY;
    double dx, dy, dt;
    const double *Ca, *Cs;                 /* [NY][NX] */
    const double *bEx, *aEx, *kiEx;        /* [NX] */
    const double *bHx, *aHx, *kiHx;        /* [NX] */
    const double *bEy, *aEy, *kiEy;        /* [NY] */
    const double *bHy, *aHy, *kiHy;        /* [NY] */
} orc_prob;

/* Ez cells updated by the E step: the outer ring stays a PEC wall. */
static int orc_e_cell(const orc_prob *p, int i, int j)
{
    return i >= 1 && i <= p->NX - 2 && j >= 1 && j <= p->NY - 2;
}

/* ------------------------------------------------------------------------ */
/* Forward sweep for one shot: steps n0 .. n0+nsteps-1 of Algorithm 1.       */
/* State (in/out): E = Ez^n, Hx/Hy = H^{n-1/2}, CPML memory psi_*.           */
/* Per step, in the order of Algorithm 1:                                    */
/*   1. record receivers: tr[n][r] = Ez^n(rec_r)                             */
/*   2-3. H half step with H-CPML (Eqs. (4), (5))                            */
/*   4-5. E step with E-CPML (Eq. (3) in the coefficient form)               */
/*   6. source: Ez(src) -= Cs(src) w[n] / (dx dy)   (Sec. 3.2, dipole kernel, */
/*      dipole length over cell depth taken as 1: w is a line current in A)   */
/*   7. save wavefield: hist[n+1-n0] = Ez^{n+1} (hist[0] = Ez^{n0})          */
/* w is indexed by absolute step n; tr and hist relative to n0.  A source   */
/* index si < 0 means no source.                                             */
/* ------------------------------------------------------------------------ */
void orc_forward_run(const orc_prob *p, double *E, double *Hx, double *Hy,
                     double *psi_hx, double *psi_hy, double *psi_ex,
                     double *psi_ey, int n0, int nsteps, int si, int sj,
                     const double *w, int nrec, const int32_t *rec_ij,
                     double *tr, double *hist)
{
    const int NX = p->NX, NY = p->NY;
    const double ch = p->dt / ORC_MU0;
    const size_t ncell = (size_t)NX * NY;
    if (hist) memcpy(hist, E, ncell * sizeof(double));

    for (int s = 0; s < nsteps; ++s) {
        const int n = n0 + s;

        /* 1. receivers see Ez^n before the step */
        if (tr) {
            for (int r = 0; r < nrec; ++r) {
                int ri = rec_ij[2 * r], rj = rec_ij[2 * r + 1];
                tr[(size_t)s * nrec + r] = E[(size_t)rj * NX + ri];
            }
        }

        /* 2-3. magnetic field and its CPML memory */
#pragma omp parallel for schedule(static)
        for (int j = 0; j < NY; ++j) {
            for (int i = 0; i < NX; ++i) {
                size_t k = (size_t)j * NX + i;
                if (j <= NY - 2) {
                    double de = (E[k + NX] - E[k]) / p->dy;
                    psi_hx[k] = p->bHy[j] * psi_hx[k] + p->aHy[j] * de;
                    Hx[k] -= ch * (de * p->kiHy[j] + psi_hx[k]);
                }
                if (i <= NX - 2) {
                    double de = (E[k + 1] - E[k]) / p->dx;
                    psi_hy[k] = p->bHx[i] * psi_hy[k] + p->aHx[i] * de;
                    Hy[k] += ch * (de * p->kiHx[i] + psi_hy[k]);
                }
            }
        }

        /* 4-5. electric field and its CPML memory */
#pragma omp parallel for schedule(static)
        for (int j = 0; j < NY; ++j) {
            for (int i = 0; i < NX; ++i) {
                if (!orc_e_cell(p, i, j)) continue;
                size_t k = (size_t)j * NX + i;
                double ddx = (Hy[k] - Hy[k - 1]) / p->dx;
                double ddy = (Hx[k] - Hx[k - NX]) / p->dy;
                psi_ex[k] = p->bEx[i] * psi_ex[k] + p->aEx[i] * ddx;
                psi_ey[k] = p->bEy[j] * psi_ey[k] + p->aEy[j] * ddy;
                E[k] = p->Ca[k] * E[k] +
                       p->Cs[k] * ((ddx * p->kiEx[i] + psi_ex[k]) -
                                   (ddy * p->kiEy[j] + psi_ey[k]));
            }
        }

        /* 6. source injection */
        if (si >= 0 && w) {
            size_t k = (size_t)sj * NX + si;
            E[k] -= p->Cs[k] * w[n] / (p->dx * p->dy);
        }

        /* 7. keep Ez^{n+1} for the adjoint */
        if (hist) memcpy(hist + (size_t)(s + 1) * ncell, E, ncell * sizeof(double));
    }
}

/* ------------------------------------------------------------------------ */
/* Adjoint sweep for one shot, n = n_hi-1 down to n_lo (Algorithm 2, as the */
/* exact transpose of one forward step; the continuous system it            */
/* discretises is Eqs. (8)-(10)).                                            */
/*                                                                           */
/* State (in/out): lE = dJ/dEz^{n+1}, lHx/lHy = dJ/dH^{n+1/2}, and the      */
/* adjoints of the CPML memories (phi_*).  On entry for n = nt-1 all zero   */
/* (terminal condition, Eq. (10)).                                           */
/*                                                                           */
/* Per step:                                                                 */
/*   A0. imaging (Eqs. (12), (13) in discrete form): for updated cells,      */
/*       S1 += lE (Ez^{n+1} - Ez^n),  S2 += lE (Ez^{n+1} + Ez^n);            */
/*       source adjoint: sadj[n] = -Cs(src) lE(src) / (dx dy)                */
/*   A1. transpose of the E step (with E-CPML)                               */
/*   A2. transpose of the H step (with H-CPML)                               */
/*   A3. adjoint source: lE(rec_r) += res[n][r]  (Alg. 2, step 1, applied    */
/*       where it enters the transposed recursion)                           */
/* hist[k] holds Ez^{k} for the shot; res is [nt][nrec] indexed by n.        */
/* ------------------------------------------------------------------------ */
void orc_adjoint_run(const orc_prob *p, double *lE, double *lHx, double *lHy,
                     double *phi_hx, double *phi_hy, double *phi_ex,
                     double *phi_ey, int n_hi, int n_lo, int si, int sj,
                     int nrec, const int32_t *rec_ij, const double *res,
                     const double *hist, double *S1, double *S2, double *sadj,
                     double *tmpx, double *tmpy)
{
    const int NX = p->NX, NY = p->NY;
    const double ch = p->dt / ORC_MU0;
    const size_t ncell = (size_t)NX * NY;

    for (int n = n_hi - 1; n >= n_lo; --n) {
        const double *En = hist + (size_t)n * ncell;
        const double *En1 = hist + (size_t)(n + 1) * ncell;

        /* A0. zero-lag cross-correlation of lE^{n+1} with the forward field */
#pragma omp parallel for schedule(static)
        for (int j = 0; j < NY; ++j) {
            for (int i = 0; i < NX; ++i) {
                if (!orc_e_cell(p, i, j)) continue;
                size_t k = (size_t)j * NX + i;
                S1[k] += lE[k] * (En1[k] - En[k]);
                S2[k] += lE[k] * (En1[k] + En[k]);
            }
        }
        if (sadj && si >= 0) {
            size_t k = (size_t)sj * NX + si;
            sadj[n] = -p->Cs[k] * lE[k] / (p->dx * p->dy);
        }

        /* A1. transpose of the E step.  The forward E step reads
         *   Ez' = Ca Ez + Cs [ (Dx/kx + psi_ex') - (Dy/ky + psi_ey') ]
         *   psi_ex' = bx psi_ex + ax Dx,  psi_ey' = by psi_ey + ay Dy
         *   Dx = (Hy(i) - Hy(i-1))/dx,    Dy = (Hx(j) - Hx(j-1))/dy.
         * With g = Cs lE', the adjoint of Dx is g/kx + ax (phi_ex + g), of Dy
         * is -g/ky + ay (phi_ey - g); the memories become bx (phi_ex + g) and
         * by (phi_ey - g); lE becomes Ca lE'.  tmpx/tmpy hold the adjoints
         * of Dx and Dy (zero outside updated cells). */
#pragma omp parallel for schedule(static)
        for (int j = 0; j < NY; ++j) {
            for (int i = 0; i < NX; ++i) {
                size_t k = (size_t)j * NX + i;
                if (!orc_e_cell(p, i, j)) {
                    tmpx[k] = 0.0;
                    tmpy[k] = 0.0;
                    continue;
                }
                double g = p->Cs[k] * lE[k];
                double tx = phi_ex[k] + g;
                double ty = phi_ey[k] - g;
                tmpx[k] = g * p->kiEx[i] + p->aEx[i] * tx;
                tmpy[k] = -g * p->kiEy[j] + p->aEy[j] * ty;
                phi_ex[k] = p->bEx[i] * tx;
                phi_ey[k] = p->bEy[j] * ty;
                lE[k] = p->Ca[k] * lE[k];
            }
        }
        /* Dx(i,j) reads Hy(i,j) with +1/dx and Hy(i-1,j) with -1/dx, so
         * lHy(i,j) gains (tmpx(i,j) - tmpx(i+1,j))/dx; likewise for Hx. */
#pragma omp parallel for schedule(static)
        for (int j = 0; j < NY; ++j) {
            for (int i = 0; i < NX; ++i) {
                size_t k = (size_t)j * NX + i;
                double ax = tmpx[k] - (i + 1 < NX ? tmpx[k + 1] : 0.0);
                double ay = tmpy[k] - (j + 1 < NY ? tmpy[k + NX] : 0.0);
                lHy[k] += ax / p->dx;
                lHx[k] += ay / p->dy;
            }
        }

        /* A2. transpose of the H step.  The forward H step reads
         *   Hx' = Hx - ch (De_y/ky + psi_hx'),  psi_hx' = by psi_hx + ay De_y
         *   Hy' = Hy + ch (De_x/kx + psi_hy'),  psi_hy' = bx psi_hy + ax De_x
         *   De_y = (Ez(j+1) - Ez(j))/dy,        De_x = (Ez(i+1) - Ez(i))/dx.
         * lHx and lHy pass through unchanged (identity in H). */
#pragma omp parallel for schedule(static)
        for (int j = 0; j < NY; ++j) {
            for (int i = 0; i < NX; ++i) {
                size_t k = (size_t)j * NX + i;
                if (j <= NY - 2) {
                    double h = ch * lHx[k];
                    double t = phi_hx[k] - h;
                    tmpy[k] = -h * p->kiHy[j] + p->aHy[j] * t;
                    phi_hx[k] = p->bHy[j] * t;
                } else {
                    tmpy[k] = 0.0;
                }
                if (i <= NX - 2) {
                    double h = ch * lHy[k];
                    double t = phi_hy[k] + h;
                    tmpx[k] = h * p->kiHx[i] + p->aHx[i] * t;
                    phi_hy[k] = p->bHx[i] * t;
                } else {
                    tmpx[k] = 0.0;
                }
            }
        }
        /* De_x(i,j) reads Ez(i+1,j) with +1/dx and Ez(i,j) with -1/dx, so
         * lE(i,j) gains (tmpx(i-1,j) - tmpx(i,j))/dx; likewise in y.  The PEC
         * ring is not a state variable: its adjoint stays zero. */
#pragma omp parallel for schedule(static)
        for (int j = 0; j < NY; ++j) {
            for (int i = 0; i < NX; ++i) {
                size_t k = (size_t)j * NX + i;
                if (!orc_e_cell(p, i, j)) {
                    lE[k] = 0.0;
                    continue;
                }
                lE[k] += (tmpx[k - 1] - tmpx[k]) / p->dx +
                         (tmpy[k - NX] - tmpy[k]) / p->dy;
            }
        }

        /* A3. adjoint source at the receivers */
        if (res) {
            for (int r = 0; r < nrec; ++r) {
                int ri = rec_ij[2 * r], rj = rec_ij[2 * r + 1];
                lE[(size_t)rj * NX + ri] += res[(size_t)n * nrec + r];
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Gradients from the accumulated correlations (Eqs. (12), (13), discrete):  */
/* with Ez^{n+1} = Ca Ez^n + Cs Q and Ca, Cs from EA, EB above,              */
/*   d Ez^{n+1} / d eps_r = -(eps0 / (dt EA)) (Ez^{n+1} - Ez^n)              */
/*   d Ez^{n+1} / d sigma = -(1 / (2 EA)) (Ez^{n+1} + Ez^n)                  */
/* so g_eps_r = -eps0/(dt EA) S1 and g_sigma = -S2/(2 EA).  Cells outside    */
/* the E update and perfect-conductor cells have constant coefficients and   */
/* get zero.                                                                 */
/* ------------------------------------------------------------------------ */
void orc_gradient_finalize(int NX, int NY, const double *eps_r,
                           const double *sigma, double dt, const double *S1,
                           const double *S2, double *g_eps, double *g_sig)
{
    for (int j = 0; j < NY; ++j) {
        for (int i = 0; i < NX; ++i) {
            size_t k = (size_t)j * NX + i;
            int upd = i >= 1 && i <= NX - 2 && j >= 1 && j <= NY - 2;
            if (!upd || sigma[k] > ORC_PEC_SIGMA) {
                g_eps[k] = 0.0;
                g_sig[k] = 0.0;
                continue;
            }
            double EA = ORC_EPS0 * eps_r[k] / dt + 0.5 * sigma[k];
            g_eps[k] = -ORC_EPS0 / (dt * EA) * S1[k];
            g_sig[k] = -S2[k] / (2.0 * EA);
        }
    }
}

/* Size of orc_prob so the Python side can allocate it opaquely. */
int orc_prob_size(void) { return (int)sizeof(orc_prob); }

void orc_prob_init(orc_prob *p, int NX, int NY, double dx, double dy,
                   double dt, const double *Ca, const double *Cs,
                   const double *bEx, const double *aEx, const double *kiEx,
                   const double *bHx, const double *aHx, const double *kiHx,
                   const double *bEy, const double *aEy, const double *kiEy,
                   const double *bHy, const double *aHy, const double *kiHy)
{
    p->NX = NX;
    p->NY = NY;
    p->dx = dx;
    p->dy = dy;
    p->dt = dt;
    p->Ca = Ca;
    p->Cs = Cs;
    p->bEx = bEx; p->aEx = aEx; p->kiEx = kiEx;
    p->bHx = bHx; p->aHx = aHx; p->kiHx = kiHx;
    p->bEy = bEy; p->aEy = aEy; p->kiEy = kiEy;
    p->bHy = bHy; p->aHy = aHy; p->kiHy = kiHy;
}
