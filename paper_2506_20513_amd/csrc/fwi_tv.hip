// Total-variation regularisation term (Sec. 3.4, Algorithm 3): a
// split-Bregman iteration of TV denoising per field, its result turned into
// the gradient term weight * (X - s U).  The operation is documented in
// include/fwi_tv.h.
//
// One launch per iteration.  Iteration t reads U_t and the multipliers
// B_{t-1} and writes B_t and U_{t+1}: the soft threshold of step 6 and the
// multiplier update of step 7 of iteration t-1 are evaluated where the
// U-update of iteration t needs them (at the cell and at its left and upper
// neighbours), so Z is never stored.  With W = D U_t + B_{t-1}:
//   Z_t = shrink(W, 1/lam),  B_t = W - Z_t,  Z_t - B_t = 2 Z_t - W.
// Memory-bound 7-point stencil over U plus 3-point reads of B; every array
// is row-major [nfield][ny][nx], one thread per cell, 64-wide rows per wave.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "fwi_tv.h"

namespace {

constexpr int kMaxBlocks = 1024;   // partial maxima per field
constexpr size_t kAlign = 256;

struct TvParams {
    float mu[FWI_TV_MAX_FIELDS];
    float lam[FWI_TV_MAX_FIELDS];
    float weight[FWI_TV_MAX_FIELDS];
};

size_t up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t u[2], bx[2], by[2], part, scale, total;
};

Layout layout(int nfield, int ny, int nx) {
    const size_t field = up((size_t)nfield * ny * nx * sizeof(float));
    Layout L;
    size_t o = 0;
    for (int k = 0; k < 2; ++k) { L.u[k] = o; o += field; }
    for (int k = 0; k < 2; ++k) { L.bx[k] = o; o += field; }
    for (int k = 0; k < 2; ++k) { L.by[k] = o; o += field; }
    L.part = o;
    o += up((size_t)nfield * kMaxBlocks * sizeof(float));
    L.scale = o;
    o += up((size_t)nfield * sizeof(float));
    L.total = o;
    return L;
}

__global__ __launch_bounds__(256) void k_absmax(const float *__restrict__ X,
                                                float *__restrict__ part, size_t n) {
    __shared__ float red[256];
    const float *x = X + (size_t)blockIdx.y * n;
    float m = 0.f;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
        m = fmaxf(m, fabsf(x[i]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)blockIdx.y * kMaxBlocks + blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_absmax_final(const float *__restrict__ part,
                                                      float *__restrict__ scale, int nb) {
    __shared__ float red[256];
    float m = 0.f;
    for (int i = threadIdx.x; i < nb; i += 256) m = fmaxf(m, part[(size_t)blockIdx.x * kMaxBlocks + i]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) scale[blockIdx.x] = red[0];
}

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// 2 shrink(w, t) - w for both components (t = 1/lam), and B = w - shrink(w, t)
__device__ __forceinline__ void bregman(float wx, float wy, float t, float &px, float &py,
                                        float &bx, float &by) {
    const float mag = sqrtf(wx * wx + wy * wy);
    const float f = mag > t ? (mag - t) / mag : 0.f;
    const float zx = wx * f, zy = wy * f;
    bx = wx - zx;
    by = wy - zy;
    px = zx - bx;
    py = zy - by;
}

__global__ __launch_bounds__(256) void k_tv_iter(
    const float *__restrict__ X, const float *__restrict__ scale, const float *__restrict__ U,
    const float *__restrict__ Bx, const float *__restrict__ By, float *__restrict__ Uo,
    float *__restrict__ Bxo, float *__restrict__ Byo, float *__restrict__ grad, int ny, int nx,
    TvParams p, int first, int last) {
    const int i = blockIdx.x * 64 + threadIdx.x;
    const int j = blockIdx.y * 4 + threadIdx.y;
    const int f = blockIdx.z;
    if (i >= nx || j >= ny) return;
    const size_t off = (size_t)f * ny * nx;
    const size_t c = off + (size_t)j * nx + i;
    const float s = scale[f];
    if (s == 0.f) {                      // all-zero field: its term is zero
        if (!last) {
            Uo[c] = 0.f;
            Bxo[c] = 0.f;
            Byo[c] = 0.f;
        }
        return;
    }
    const float inv = 1.f / s, mu = p.mu[f], lam = p.lam[f];
    const int im = wrap(i - 1, nx), ip = wrap(i + 1, nx), jm = wrap(j - 1, ny), jp = wrap(j + 1, ny);
    const float *src = first ? X : U;
    const float sc = first ? inv : 1.f;  // U_0 = X / s
    auto u = [&](int jj, int ii) { return src[off + (size_t)jj * nx + ii] * sc; };
    const float uc = u(j, i), ul = u(j, im), ur = u(j, ip), uu = u(jm, i), ud = u(jp, i);
    float pcx = 0.f, pcy = 0.f, plx = 0.f, puy = 0.f, bcx = 0.f, bcy = 0.f;
    if (!first) {
        const float t = 1.f / lam;
        float dum0, dum1, qx, qy;
        // at (j, i)
        bregman(ur - uc + Bx[c], ud - uc + By[c], t, pcx, pcy, bcx, bcy);
        // at (j, i-1): needs U(j+1, i-1)
        const size_t cl = off + (size_t)j * nx + im;
        bregman(uc - ul + Bx[cl], u(jp, im) - ul + By[cl], t, plx, qy, dum0, dum1);
        // at (j-1, i): needs U(j-1, i+1)
        const size_t cu = off + (size_t)jm * nx + i;
        bregman(u(jm, ip) - uu + Bx[cu], uc - uu + By[cu], t, qx, puy, dum0, dum1);
        (void)qx;
        (void)qy;
    }
    if (!last) {
        Bxo[c] = bcx;
        Byo[c] = bcy;
    }
    const float dtp = -((pcx - plx) + (pcy - puy));           // D^T (Z - B)
    const float xn = X[c] * inv;
    const float un = (mu * xn + lam * dtp + lam * (4.f * uc + ul + ur + uu + ud)) / (mu + 8.f * lam);
    if (last)
        grad[c] += p.weight[f] * (X[c] - s * un);
    else
        Uo[c] = un;
}

}  // namespace

extern "C" {

size_t fwi_tv_workspace_bytes(int32_t nfield, int32_t ny, int32_t nx) {
    if (nfield < 1 || nfield > FWI_TV_MAX_FIELDS || ny < 2 || nx < 2 ||
        (int64_t)ny * nx >= ((int64_t)1 << 31))
        return 0;
    return layout(nfield, ny, nx).total;
}

int fwi_tv_gradient(const float *X, float *grad, int32_t nfield, int32_t ny, int32_t nx,
                    const float *mu, const float *lam, const float *weight, int32_t iters,
                    void *ws, size_t ws_bytes, void *stream) {
    if (!X || !grad || !mu || !lam || !weight || nfield < 1 || nfield > FWI_TV_MAX_FIELDS ||
        ny < 2 || nx < 2 || (int64_t)ny * nx >= ((int64_t)1 << 31) || iters < 1)
        return -1;
    TvParams p{};
    for (int f = 0; f < nfield; ++f) {
        if (!(mu[f] > 0.f) || !(lam[f] > 0.f)) return -1;
        p.mu[f] = mu[f];
        p.lam[f] = lam[f];
        p.weight[f] = weight[f];
    }
    const Layout L = layout(nfield, ny, nx);
    if (!ws || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0 || ws_bytes < L.total) return -4;
    char *w = static_cast<char *>(ws);
    auto F = [&](size_t o) { return reinterpret_cast<float *>(w + o); };
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t n = (size_t)ny * nx;
    const int nb = (int)std::min<size_t>(kMaxBlocks, (n + 255) / 256);
    hipLaunchKernelGGL(k_absmax, dim3(nb, nfield), dim3(256), 0, st, X, F(L.part), n);
    hipLaunchKernelGGL(k_absmax_final, dim3(nfield), dim3(256), 0, st, F(L.part), F(L.scale), nb);
    const dim3 grid((nx + 63) / 64, (ny + 3) / 4, nfield), block(64, 4);
    for (int t = 0; t < iters; ++t) {
        const int first = t == 0, last = t == iters - 1;
        hipLaunchKernelGGL(k_tv_iter, grid, block, 0, st, X, F(L.scale), F(L.u[t & 1]),
                           F(L.bx[(t + 1) & 1]), F(L.by[(t + 1) & 1]), F(L.u[(t + 1) & 1]),
                           F(L.bx[t & 1]), F(L.by[t & 1]), grad, ny, nx, p, first, last);
    }
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

}  // extern "C"
