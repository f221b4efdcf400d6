// Internal declarations of the FWI library: problem dimensions, workspace
// layout and kernel argument blocks.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace fwi {

// Physical constants (Sec. 2.1: mu is the free-space permeability).
constexpr double kPi = 3.14159265358979323846;
constexpr double kC0 = 299792458.0;
constexpr double kMu0 = 4.0e-7 * kPi;
constexpr double kEps0 = 1.0 / (kMu0 * kC0 * kC0);
// Conductivity above which a cell is a perfect conductor (Sec. 3.2).
constexpr double kPecSigma = 100.0;

constexpr size_t kAlign = 256;
constexpr int kMisfitBlocks = 512;

// Problem dimensions after validation.
struct Dims {
    int NX, NY;        // total grid
    int npml, nt;
    int S, R;          // shots, receivers per shot
    int pitch;         // floats per field row (NX rounded up to 64)
    int W;             // width of the x-direction CPML strip store (2 npml + 1)
    int Hs;            // height of the y-direction CPML strip store (2 npml + 1)
    size_t plane;      // NY * pitch, one shot's field
    size_t xs;         // NY * W, one shot's x-strip store
    size_t ys;         // Hs * pitch, one shot's y-strip store
    double dx, dy, dt;
    int cpml_order;
    double cpml_sigma_scale, cpml_kappa_max, cpml_alpha_max;
};

// CPML profiles as float arrays in the workspace.  x arrays have NX entries,
// y arrays NY entries.  b, a and 1/kappa at E (integer) and H (half-integer)
// positions.
struct Profiles {
    float *bEx, *aEx, *kEx, *bHx, *aHx, *kHx;
    float *bEy, *aEy, *kEy, *bHy, *aHy, *kHy;
};

// Field state of all shots.  For the forward state E lives in the E slots
// (history / segment buffer) and `E` is unused.  The four CPML memories are
// stored only in their strips:
//   phx (psi of Hx, y-derivative) and pey (psi of Ez, y-derivative):
//       [S][Hs][pitch], row r <-> j = r (r < npml) or NY-1-npml + (r-npml)
//   phy (psi of Hy, x-derivative) and pex (psi of Ez, x-derivative):
//       [S][NY][W],     col c <-> i = c (c < npml) or NX-1-npml + (c-npml)
struct State {
    float *E, *Hx, *Hy, *phx, *phy, *pex, *pey;
};

struct Layout {
    Dims d;
    int mode;          // FWI_SAVE_* or -1 for fwi_gradient
    int K;             // checkpoint interval (checkpoint modes)
    int ncp;           // number of checkpoints
    int nslots;        // Ez slots
    size_t off_Ca, off_Cs, off_prof;
    size_t off_src, off_rec, off_rord, off_rlen;
    size_t off_fwd[2];
    size_t off_slots;
    size_t off_ckpt, ckpt_stride;
    size_t off_adj[2];
    size_t off_S1, off_S2;
    size_t off_res, off_trc, off_mis;
    size_t state_bytes;   // one forward State (without E)
    size_t total;
};

// ---- kernel argument blocks -------------------------------------------------

struct StepGeom {
    const int *src_ij;        // device [S][2]
    const float *wavelet;     // device [S][nt]
    const int *rec_ij;        // device [S][R][2]
    float *traces;            // device [S][nt][R] or null (no recording)
};

struct FwdStepArgs {
    int NX, NY, npml, pitch, W, Hs, S, R, nt, n;
    size_t plane, xs, ys;
    float rdx, rdy, ch, src_scale;
    const float *Ca, *Cs;
    Profiles p;
    const float *E_in;
    float *E_out;
    State in, out;
    StepGeom g;
};

struct AdjStepArgs {
    int NX, NY, npml, pitch, W, Hs, S, R, nt, n;
    size_t plane, xs, ys;
    float rdx, rdy, ch, src_scale;
    const float *Ca, *Cs;
    Profiles p;
    const float *E_np1;       // forward Ez^{n+1}, all shots
    const float *E_n;         // forward Ez^n
    State in, out;            // adjoint state lambda^{n+1} -> lambda^n
    float *S1, *S2;           // [NY][pitch] correlation accumulators
    const int *src_ij;
    float *src_adjoint;       // [S][nt] or null
};

// ---- launchers (fwi_kernels.hip) ------------------------------------------

hipError_t launch_coefficients(const float *eps_r, const float *sigma, float *Ca,
                               float *Cs, int NX, int NY, int pitch, double dt,
                               hipStream_t st);
hipError_t launch_profiles(const Dims &d, const Profiles &p, hipStream_t st);
hipError_t launch_fill(float *dst, size_t n, float v, hipStream_t st);
hipError_t launch_fwd_step(const FwdStepArgs &a, hipStream_t st);
hipError_t launch_adj_step(const AdjStepArgs &a, hipStream_t st);
hipError_t launch_adj_inject(const float *residual, float *lE, const int *rec_ij,
                             const int *order, const int *glen, int S, int R,
                             int nt, int n, size_t plane, int pitch,
                             hipStream_t st);
hipError_t launch_gradient_finalize(const float *eps_r, const float *sigma,
                                    const float *S1, const float *S2,
                                    float *g_eps, float *g_sig, int NX, int NY,
                                    int pitch, double dt, hipStream_t st);
hipError_t launch_residual_misfit(const float *traces, const float *observed,
                                  float *residual, size_t n, double *partials,
                                  double *misfit, hipStream_t st);

}  // namespace fwi
