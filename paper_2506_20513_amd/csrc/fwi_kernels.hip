// HIP kernels for gfx950 around the stencil: update coefficients, CPML
// profiles, fills, gradient scaling and the misfit reduction.  The stencil
// kernels themselves are in fwi_stream.hip.
//
// Paper: arXiv 2506.20513, Sec. 2.1 (Eqs. (6), (12), (13)), Sec. 3.2.
//
// Layout: every field of every shot is a [NY][pitch] plane (x contiguous,
// pitch = NX rounded up to 64 floats), shots stacked [S][NY][pitch].
#include "fwi_internal.h"

#include <math.h>

namespace fwi {
namespace {

__device__ __forceinline__ bool ecell(int i, int j, int NX, int NY) {
    return i >= 1 && i <= NX - 2 && j >= 1 && j <= NY - 2;
}

// ---------------------------------------------------------------------------
// Update coefficients, double precision, stored as float (Sec. 3.2,
// coefficient kernel): Ca = EB/EA, Cs = 1/EA; sigma > 100 S/m => 0.  The
// PEC ring, which the E step never updates, also gets 0: the stencil kernels
// then need no per-cell predicate (its Ez stays exactly 0).
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
    if (ecell(i, j, NX, NY) && !(sg > kPecSigma)) {
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

// Merged copies: block b copies floats [b C, (b + 1) C) of the entries laid
// end to end, starting from the entry its first float falls in (binary
// search over the prefix sums) and moving on to the next entries.
constexpr unsigned long long kCopyChunk = 8192;

__global__ __launch_bounds__(256) void k_copy_table(const CopyEntry *__restrict__ tab,
                                                    const unsigned long long *__restrict__ cum,
                                                    int nent, unsigned long long total) {
    const unsigned long long beg = (unsigned long long)blockIdx.x * kCopyChunk;
    const unsigned long long end = beg + kCopyChunk < total ? beg + kCopyChunk : total;
    int lo = 0, hi = nent - 1;            // the last entry with cum[e] <= beg
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (cum[mid] <= beg)
            lo = mid;
        else
            hi = mid - 1;
    }
    for (int e = lo; e < nent && cum[e] < end; ++e) {
        const unsigned long long c0 = cum[e];
        const unsigned long long a = beg > c0 ? beg : c0;
        const unsigned long long b = end < cum[e + 1] ? end : cum[e + 1];
        float *dst = tab[e].dst;
        const float *src = tab[e].src;
        for (unsigned long long i = a + threadIdx.x; i < b; i += blockDim.x) dst[i - c0] = src[i - c0];
    }
}

// Shot sums of the correlations, in shot order and double precision, then
// g_eps = -eps0/(dt EA) S1, g_sig = -S2/(2 EA) on updated, non-PEC cells.
__global__ void k_gradient_finalize(const float *__restrict__ eps_r,
                                    const float *__restrict__ sigma,
                                    const float *__restrict__ S1,
                                    const float *__restrict__ S2, int S, size_t plane,
                                    float *__restrict__ ge, float *__restrict__ gs,
                                    int NX, int NY, int pitch, double dt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= NX || j >= NY) return;
    const size_t o = (size_t)j * NX + i;
    const size_t k = (size_t)j * pitch + i;
    float a = 0.f, b = 0.f;
    const double sg = sigma[o];
    if (ecell(i, j, NX, NY) && !(sg > kPecSigma)) {
        double s1 = 0.0, s2 = 0.0;
        for (int s = 0; s < S; ++s) {
            s1 += (double)S1[(size_t)s * plane + k];
            s2 += (double)S2[(size_t)s * plane + k];
        }
        const double EA = kEps0 * (double)eps_r[o] / dt + 0.5 * sg;
        a = (float)(-kEps0 / (dt * EA) * s1);
        b = (float)(-s2 / (2.0 * EA));
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

// FP64 sums of squares of two float arrays (the gradient-norm reduction),
// per-block partials in a fixed order.  A sum is non-finite exactly when an
// element is: the square of any finite float fits a double many times over.
__global__ __launch_bounds__(256) void k_sumsq2(const float *__restrict__ a, size_t na,
                                                const float *__restrict__ b, size_t nb,
                                                double *__restrict__ partials) {
    __shared__ double red[256];
    double acc = 0.0;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t t0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (size_t t = t0; t < na; t += stride) acc += (double)a[t] * (double)a[t];
    for (size_t t = t0; t < nb; t += stride) acc += (double)b[t] * (double)b[t];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

// flag = 1 if the summed partials, or the optional scalar, are not finite.
__global__ __launch_bounds__(256) void k_finite_flag(const double *__restrict__ partials,
                                                     int np, const double *__restrict__ scalar,
                                                     int *__restrict__ flag) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int t = threadIdx.x; t < np; t += 256) acc += partials[t];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        bool bad = !isfinite(red[0]);
        if (scalar) bad = bad || !isfinite(*scalar);
        *flag = bad ? 1 : 0;
    }
}

}  // namespace

hipError_t launch_finite_check(const float *a, size_t na, const float *b, size_t nb,
                               const double *scalar, double *partials, int *flag,
                               hipStream_t st) {
    hipLaunchKernelGGL(k_sumsq2, dim3(kMisfitBlocks), dim3(256), 0, st, a, na, b, nb,
                       partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_finite_flag, dim3(1), dim3(256), 0, st, partials, kMisfitBlocks,
                       scalar, flag);
    return hipGetLastError();
}

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

hipError_t launch_copy_table(const CopyEntry *tab, const unsigned long long *cum, int nent,
                             unsigned long long total, hipStream_t st) {
    if (total == 0 || nent < 1) return hipSuccess;
    const unsigned long long blocks = (total + kCopyChunk - 1) / kCopyChunk;
    if (blocks > 0x7fffffffull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_copy_table, dim3((unsigned)blocks), dim3(256), 0, st, tab, cum, nent,
                       total);
    return hipGetLastError();
}

hipError_t launch_gradient_finalize(const float *eps_r, const float *sigma,
                                    const float *S1, const float *S2, int S,
                                    size_t plane, float *g_eps, float *g_sig, int NX,
                                    int NY, int pitch, double dt, hipStream_t st) {
    hipLaunchKernelGGL(k_gradient_finalize, dim3((NX + 255) / 256, NY), dim3(256), 0,
                       st, eps_r, sigma, S1, S2, S, plane, g_eps, g_sig, NX, NY, pitch, dt);
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
