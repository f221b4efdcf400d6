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
    int depth;         // temporal depth of the streaming passes
    int ncp;           // number of checkpoints
    int nslots;        // Ez slots
    // streaming decomposition (see Tiling): row bands of the forward kernel
    // and, chosen for its own occupancy, of the adjoint kernel
    int nstrip, nband, naband;
    int bands[64];
    int abands[64];
    size_t off_Ca, off_Cs, off_prof;
    size_t off_src, off_rrow, off_rcol, off_ridx, off_rspan, off_bands, off_abands, off_cold;
    size_t off_fwd[2];
    size_t off_slots;
    size_t off_ckpt, ckpt_stride;
    size_t off_adj[2];
    size_t off_S1, off_S2;    // per-shot [S][NY][pitch]
    size_t off_res, off_trc, off_mis;
    size_t off_chk;       // finiteness check: kMisfitBlocks partials, then the flag
    size_t state_bytes;   // one forward State (without E)
    size_t total;
};

// ---- kernel argument blocks -------------------------------------------------

// Time levels advanced per pass of the streaming kernels (temporal depth).
// Depth 8 reads and writes each field row once per 8 steps, but the
// dependency cone leaves a 64-lane strip 48 output columns (16 recomputed)
// and the kernels need 110-165 VGPRs; depth 4 keeps 56 columns and 75-100
// VGPRs.  Measured: depth 8 gives 45% more cell-updates per second on a
// 2088x1064 grid with 64 shots (300 against 207 G/s), and was 12-38% slower
// on grids of 0.02-0.25 M cells, where the longer pipeline start of every
// band weighs more.  A problem uses depth 8 from kDepthLargeCells cells per
// shot on.  A batch of problems runs all its merged passes at one depth:
// depth 4 unless its plan's autotuner (or its caller) picks depth 8.
constexpr int kDepthSmall = 4;
constexpr int kDepthLarge = 8;
constexpr long long kDepthLargeCells = 1LL << 20;

// Source and receiver tables on the device.  Receivers of each shot are
// sorted by (row, column), stable in receiver index; rrow is the row CSR.
struct StreamGeom {
    const int *src_ij;        // [S][2]
    const float *wavelet;     // [S][nt]
    const int *rrow;          // [S][NY+1]
    const int *rcol;          // [S][R] column of the q-th receiver in that order
    const int *ridx;          // [S][R] its receiver index
    const int *rspan;         // [S][2] first and last receiver row
};

// Streaming decomposition: nstrip x-strips of 64 - 2K output columns and
// nband row bands; bands[b] .. bands[b+1] are the rows a wave of band b owns.
struct Tiling {
    const int *bands;         // [nband + 1]
    int nstrip, nband;
    int depth;                // temporal depth: kDepthSmall or kDepthLarge
};

// Per-call constants of the stencil kernels that only rare branches read
// (CPML rows and columns, receiver rows, the source row).  It lives in the
// workspace, so the kernels load these pointers only where they need them
// instead of holding them in scalar registers for the whole sweep.
struct StreamCold {
    Profiles p;
    State fs[2];              // forward H / CPML states (E unused)
    State as[2];              // adjoint states
    StreamGeom g;
    float *traces;            // [S][nt][R] or null
    const float *residual;    // [S][nt][R]
    float *src_adjoint;       // [S][nt] or null
};

// Hot arguments of one forward pass: steps n .. n+nlev-1.
struct FwdStreamArgs {
    int NX, NY, npml, pitch, W, S, R, nt;
    int n, nlev;              // first step of the pass, steps in the pass (<= K)
    int cur;                  // input state cold->fs[cur], output fs[cur ^ 1]
    int record;               // write traces
    Tiling tl;
    size_t plane, xs, ys, lev_stride;
    float ch, rdx, rdy, src_scale;
    const float *Ca, *Cs;
    const float *E_in;        // Ez^n, all shots
    float *E_out;             // Ez^{n+nlev} (unused when E_lev is set)
    float *E_lev;             // or null: Ez^{n+l+1} to E_lev + l * lev_stride
    const float *Hx_in, *Hy_in;
    float *Hx_out, *Hy_out;
    const StreamCold *cold;
};

// Hot arguments of one adjoint pass: steps n_top-1 .. n_top-nlev.
struct AdjStreamArgs {
    int NX, NY, npml, pitch, W, S, R, nt;
    int n_top, n_base, nlev;
    int cur;                  // input state cold->as[cur], output as[cur ^ 1]
    Tiling tl;
    size_t plane, xs, ys, lev_stride;
    float ch, rdx, rdy, src_scale;
    const float *Ca, *Cs;
    const float *E_lev;       // forward Ez^{n_base + k} at E_lev + k * lev_stride
    const float *L_in, *LHx_in, *LHy_in;
    float *L_out, *LHx_out, *LHy_out;
    float *S1, *S2;           // per-shot correlation sums [S][NY][pitch]
    const StreamCold *cold;
};

// ---- launchers ---------------------------------------------------------------

hipError_t launch_coefficients(const float *eps_r, const float *sigma, float *Ca,
                               float *Cs, int NX, int NY, int pitch, double dt,
                               hipStream_t st);
hipError_t launch_profiles(const Dims &d, const Profiles &p, hipStream_t st);
hipError_t launch_fill(float *dst, size_t n, float v, hipStream_t st);
// One device-to-device copy of n floats; the batched plans merge the
// checkpoint copies of every problem at one schedule position into one
// launch over a table of these.
struct CopyEntry {
    float *dst;
    const float *src;
    unsigned long long n;
};
// Copies every entry of tab (device, nent entries); cum (device, nent + 1
// values) holds the prefix sums of the entries' n, cum[nent] = total.  The
// entries must not overlap one another.
hipError_t launch_copy_table(const CopyEntry *tab, const unsigned long long *cum, int nent,
                             unsigned long long total, hipStream_t st);
hipError_t launch_gradient_finalize(const float *eps_r, const float *sigma,
                                    const float *S1, const float *S2, int S,
                                    size_t plane, float *g_eps, float *g_sig, int NX,
                                    int NY, int pitch, double dt, hipStream_t st);
hipError_t launch_residual_misfit(const float *traces, const float *observed,
                                  float *residual, size_t n, double *partials,
                                  double *misfit, hipStream_t st);
// Sets *flag (device int) to 1 if a[0..na) or b[0..nb) holds a NaN or an
// infinity, or if *scalar (device, may be null) is not finite; else 0.
// partials: kMisfitBlocks doubles of scratch.
hipError_t launch_finite_check(const float *a, size_t na, const float *b, size_t nb,
                               const double *scalar, double *partials, int *flag,
                               hipStream_t st);
// streaming kernels (fwi_stream.hip)
hipError_t launch_fwd_stream(const FwdStreamArgs &a, hipStream_t st);
hipError_t launch_adj_stream(const AdjStreamArgs &a, hipStream_t st);
// Blocks one problem's pass launches.
unsigned stream_blocks(int S, const Tiling &tl);
// One pass for nm problems at once: tab[m] (device) holds problem m's
// arguments and boff[0..nm] (device) the prefix sums of their block counts,
// nblocks = boff[nm].  depth: the passes' temporal depth (kDepthSmall or
// kDepthLarge, the same for every problem of the launch); tail: the
// problems advance fewer than depth levels.  lev (forward only): 1 if every
// problem's entry has E_lev set (segment re-forward), 0 if none has.
hipError_t launch_fwd_table(const FwdStreamArgs *tab, const unsigned *boff, int nm,
                            unsigned nblocks, int depth, bool tail, int lev, hipStream_t st);
hipError_t launch_adj_table(const AdjStreamArgs *tab, const unsigned *boff, int nm,
                            unsigned nblocks, int depth, bool tail, hipStream_t st);

}  // namespace fwi
