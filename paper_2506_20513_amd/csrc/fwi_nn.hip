// Kernels of the learned gradient preconditioner: a small encoder-decoder
// CNN with 3x3 convolutions on BF16 activations and weights, FP32
// accumulation on the gfx950 matrix cores (v_mfma_f32_16x16x32_bf16).
//
// Layouts: activations NHWC [N][H][W][C] bf16 with C a multiple of 32;
// weights [Co][3][3][Ci] bf16 (FP32 masters held by the optimiser); all
// convolutions are 3x3, stride 1, zero padding 1.
//
// MFMA 16x16x32 operand layout (lane l of the wave): A holds row l%16,
// columns 8*(l/16) .. +7; B holds rows 8*(l/16) .. +7 of column l%16; the
// 16x16 result holds rows 4*(l/16) .. +3 of column l%16.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fwi_nn.h"

namespace {

using bf16 = __bf16;
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// floor(n / d) for n d < 2^32 as the high word of n m with
// m = floor((2^32 - 1) / d) + 1 = 2^32 / d + e, 0 < e <= 1.  Then n m / 2^32 =
// n / d + n e / 2^32 with n e / 2^32 <= n / 2^32 < 1 / d, less than the
// distance from n / d up to the next integer, so the floor is exact.  d = 1
// (where m would overflow) is passed through.  The convolution kernels use
// it with d = H or W <= 2^15 (checked by the host) and n < 2 d + 2^8.
struct SmallDiv {
    unsigned d, m;
    __device__ explicit SmallDiv(unsigned dd) : d(dd), m(dd > 1 ? 0xffffffffu / dd + 1u : 0u) {}
    __device__ __forceinline__ unsigned div(unsigned n) const { return d > 1 ? __umulhi(n, m) : n; }
    __device__ __forceinline__ unsigned mod(unsigned n) const { return n - d * div(n); }
};

// y = act(conv3x3(x, w) + bias) as an implicit GEMM: rows are output pixels
// in flattened (n, y, x) order, columns output channels, the reduction runs
// over (ky, kx, ci).  Tiling over flattened pixels keeps every lane busy on
// images narrower than a tile.  This form, with operands read straight from
// global memory, serves layers too small for the LDS-tiled kernel below: a
// block of four waves covers 64 * MT consecutive pixels; wave w owns MT
// tiles of 16 pixels times 16 * NT output channels.  A tap at
// (ky, kx) reads pixel p + (ky - 1) W + (kx - 1) when it lies in the image.
template <int NT, int MT>
__global__ __launch_bounds__(256) void k_conv3x3(const bf16 *__restrict__ x,
                                                 const bf16 *__restrict__ w,
                                                 const float *__restrict__ bias,
                                                 bf16 *__restrict__ y, int N, int H, int W,
                                                 int Ci, int Co, int relu) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t P = (int64_t)N * H * W;
    const int64_t base = ((int64_t)blockIdx.x * 4 + wave) * (16 * MT);
    const int co0 = blockIdx.y * (16 * NT);
    const int kq = (lane >> 4) * 8;
    int py[MT], px[MT];
    int64_t pp[MT];
    bool pv[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        const int64_t p = base + m * 16 + (lane & 15);
        pv[m] = p < P;
        pp[m] = pv[m] ? p : 0;
        px[m] = (int)(pp[m] % W);
        py[m] = (int)((pp[m] / W) % H);
    }
    f32x4 acc[MT][NT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[m][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bf16x8 zero{};
    for (int ky = 0; ky < 3; ++ky) {
        for (int kx = 0; kx < 3; ++kx) {
            const int64_t shift = (int64_t)(ky - 1) * W + (kx - 1);
            const bf16 *xp[MT];
            bool ok[MT];
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                const int yy = py[m] + ky - 1, xx = px[m] + kx - 1;
                ok[m] = pv[m] && yy >= 0 && yy < H && xx >= 0 && xx < W;
                // out-of-image taps read a valid address and are zeroed
                xp[m] = x + (ok[m] ? (pp[m] + shift) * Ci : 0) + kq;
            }
            const bf16 *wp = w + ((size_t)(co0 + (lane & 15)) * 9 + ky * 3 + kx) * Ci + kq;
            for (int c0 = 0; c0 < Ci; c0 += 32) {
                bf16x8 a[MT];
#pragma unroll
                for (int m = 0; m < MT; ++m) {
                    a[m] = *reinterpret_cast<const bf16x8 *>(xp[m] + c0);
                    if (!ok[m]) a[m] = zero;
                }
#pragma unroll
                for (int j = 0; j < NT; ++j) {
                    const bf16x8 bv =
                        *reinterpret_cast<const bf16x8 *>(wp + (size_t)j * 16 * 9 * Ci + c0);
#pragma unroll
                    for (int m = 0; m < MT; ++m) acc[m][j] = mfma(a[m], bv, acc[m][j]);
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        const int co = co0 + 16 * j + (lane & 15);
        const float bb = bias ? bias[co] : 0.f;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t po = base + m * 16 + 4 * (lane >> 4) + r;
                if (po < P) {
                    float v = acc[m][j][r] + bb;
                    if (relu) v = fmaxf(v, 0.f);
                    y[po * Co + co] = (bf16)v;
                }
            }
        }
    }
}

// The same convolution with both operand tiles staged in LDS: a block
// computes BM (128 or 64) consecutive (flattened) pixels x BN output
// channels.  A reduction step covers one kernel row ky and 32 input channels
// for all three kx taps: it stages the input rows of pixels base - 1 ..
// base + BM shifted by ky - 1 image rows (BM + 2 rows, zero where that row
// leaves the image) and the three BN x 32 weight tiles of (ky, kx = 0, 1, 2).
// Tap kx of output pixel p reads staged row p - base + kx, so the three taps
// share the staged rows; a tap that would wrap across a row edge (kx = 0 at
// column 0, kx = 2 at column W-1) gets a zero fragment.  Two LDS buffers, one
// barrier per step; the global loads of step k+1 are in flight while step k
// issues its 3 x (BM / 64) x BN/16 MFMAs per wave.  The 64-pixel tile
// doubles the blocks of layers with few pixels, where one block per CU
// leaves every global-load latency exposed.
constexpr int kTP = 40;      // LDS row pitch in bf16: 32 channels + 8 padding (80 bytes)

template <int BN, int BM>
__global__ __launch_bounds__(256) void k_conv3x3_lds(const bf16 *__restrict__ x,
                                                     const bf16 *__restrict__ w,
                                                     const float *__restrict__ bias,
                                                     bf16 *__restrict__ y, int N, int H, int W,
                                                     int Ci, int Co, int relu) {
    static_assert(BM == 64 || BM == 128, "64 or 128 pixels per block");
    constexpr int AR = BM + 2, NTL = BN / 16, MW = BM / 64;   // MW: 16-pixel tiles per wave
    constexpr int APieces = AR * 4, BPieces = 3 * BN * 4;     // 16-byte pieces per step
    constexpr int AU = (APieces + 255) / 256, BU = (BPieces + 255) / 256;
    __shared__ __attribute__((aligned(16))) bf16 As[2][AR * kTP];
    __shared__ __attribute__((aligned(16))) bf16 Bs[2][3 * BN * kTP];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t P = (int64_t)N * H * W;
    const int64_t base = (int64_t)blockIdx.x * BM;
    const int co0 = blockIdx.y * BN;
    const int col0 = (int)(base % W), row0 = (int)((base / W) % H);
    const int nck = Ci / 32, K = 3 * nck;
    const SmallDiv dW((unsigned)W), dH((unsigned)H);
    // this lane's output pixels (offsets in the block) and their columns
    int pofs[MW], pcol[MW];
#pragma unroll
    for (int m = 0; m < MW; ++m) {
        pofs[m] = wave * 16 * MW + m * 16 + (lane & 15);
        pcol[m] = (int)dW.mod((unsigned)(col0 + pofs[m]));
    }
    uint4 ra[AU], rb[BU];
    auto fetch = [&](int k) {
        const int ky = k / nck, c0 = (k - ky * nck) * 32;
#pragma unroll
        for (int u = 0; u < AU; ++u) {
            const int idx = t + 256 * u;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (idx < APieces) {
                const int j = idx >> 2, c = (idx & 3) * 8;
                const int64_t q = base - 1 + j;
                if (q >= 0 && q < P) {
                    const int d = col0 - 1 + j;                 // >= -1
                    const int row = row0 + (d >= 0 ? (int)dW.div((unsigned)d) : -1);
                    const int yy = (int)dH.mod((unsigned)(row + H)) + ky - 1;
                    if (yy >= 0 && yy < H)
                        v = *reinterpret_cast<const uint4 *>(
                            x + (q + (int64_t)(ky - 1) * W) * Ci + c0 + c);
                }
            }
            ra[u] = v;
        }
#pragma unroll
        for (int u = 0; u < BU; ++u) {
            const int idx = t + 256 * u;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (idx < BPieces) {
                const int kx = idx / (BN * 4), r = idx - kx * (BN * 4);
                const int n = r >> 2, c = (r & 3) * 8;
                v = *reinterpret_cast<const uint4 *>(
                    w + ((size_t)(co0 + n) * 9 + ky * 3 + kx) * Ci + c0 + c);
            }
            rb[u] = v;
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int u = 0; u < AU; ++u) {
            const int idx = t + 256 * u;
            if (idx < APieces)
                *reinterpret_cast<uint4 *>(&As[buf][(idx >> 2) * kTP + (idx & 3) * 8]) = ra[u];
        }
#pragma unroll
        for (int u = 0; u < BU; ++u) {
            const int idx = t + 256 * u;
            if (idx < BPieces)
                *reinterpret_cast<uint4 *>(&Bs[buf][(idx >> 2) * kTP + (idx & 3) * 8]) = rb[u];
        }
    };
    f32x4 acc[MW][NTL];
#pragma unroll
    for (int m = 0; m < MW; ++m)
#pragma unroll
        for (int n = 0; n < NTL; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bf16x8 zero{};
    fetch(0);
    stash(0);
    __syncthreads();
    for (int k = 0; k < K; ++k) {
        const int buf = k & 1;
        if (k + 1 < K) fetch(k + 1);
#pragma unroll
        for (int kx = 0; kx < 3; ++kx) {
            bf16x8 a[MW];
#pragma unroll
            for (int m = 0; m < MW; ++m) {
                a[m] = *reinterpret_cast<const bf16x8 *>(
                    &As[buf][(pofs[m] + kx) * kTP + 8 * (lane >> 4)]);
                if ((kx == 0 && pcol[m] == 0) || (kx == 2 && pcol[m] == W - 1)) a[m] = zero;
            }
#pragma unroll
            for (int n = 0; n < NTL; ++n) {
                const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(
                    &Bs[buf][(kx * BN + n * 16 + (lane & 15)) * kTP + 8 * (lane >> 4)]);
#pragma unroll
                for (int m = 0; m < MW; ++m) acc[m][n] = mfma(a[m], bv, acc[m][n]);
            }
        }
        if (k + 1 < K) stash(buf ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int n = 0; n < NTL; ++n) {
        const int co = co0 + n * 16 + (lane & 15);
        const float bb = bias ? bias[co] : 0.f;
#pragma unroll
        for (int m = 0; m < MW; ++m) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t po = base + wave * 16 * MW + m * 16 + 4 * (lane >> 4) + r;
                if (po < P) {
                    float v = acc[m][n][r] + bb;
                    if (relu) v = fmaxf(v, 0.f);
                    y[po * Co + co] = (bf16)v;
                }
            }
        }
    }
}

// wf[ci][ky][kx][co] = w[co][2-ky][2-kx][ci]: the weights of the transposed
// convolution (input gradient = conv3x3(output gradient, wf)).
__global__ void k_flip(const bf16 *__restrict__ w, bf16 *__restrict__ wf, int Ci, int Co) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= Co * 9 * Ci) return;
    const int ci = t % Ci, k = (t / Ci) % 9, co = t / (9 * Ci);
    const int ky = k / 3, kx = k % 3;
    wf[((size_t)ci * 9 + (2 - ky) * 3 + (2 - kx)) * Co + co] = w[t];
}

// Several layers at once (one launch for the whole network): thread e writes
// element e of wf when it lies in a layer, reading the matching weight of
// w, so that the writes are coalesced.
constexpr int kFlipMax = 32;
struct FlipTable {
    int n;
    int64_t off[kFlipMax];
    int32_t ci[kFlipMax], co[kFlipMax];
};

__global__ void k_flip_layers(const bf16 *__restrict__ w, bf16 *__restrict__ wf, FlipTable tb,
                              int64_t end) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= end) return;
    for (int l = 0; l < tb.n; ++l) {
        const int64_t d = e - tb.off[l];
        const int Ci = tb.ci[l], Co = tb.co[l];
        if (d >= 0 && d < (int64_t)9 * Ci * Co) {
            const int dd = (int)d;
            const int co = dd % Co, k = (dd / Co) % 9, ci = dd / (9 * Co);
            wf[e] = w[tb.off[l] + ((int64_t)co * 9 + (8 - k)) * Ci + ci];
            return;
        }
    }
}

// ---------------------------------------------------------------------------
// Weight and bias gradients: dw[co][ky][kx][ci] = sum_q dz[q][co] x[q + (ky-1, kx-1)][ci],
// db[co] = sum_q dz[q][co].  A GEMM whose reduction runs over output pixels
// q: a block owns a 32 (co) x 32 (ci) tile for all nine taps, loops over
// every gridDim.x-th chunk of CH pixels and writes its partial sums to
// record blockIdx.x of part (Co 9 Ci weight sums, then Co bias sums).
//
// Per chunk q0 .. q0+CH-1 the block stages, in natural (pixel-major) layout:
//   Z[j][c]      = dz[q0 + j][co tile]                          (CH rows)
//   X[ky][j][c]  = x[q0 - 1 + j + (ky-1) W][ci tile]             (CH + 2 rows)
// and each wave runs nine MFMAs per 32 pixels of the chunk.  Chunks of 64
// pixels (half the barriers and staging rounds per MFMA) made the training
// step 4% slower than chunks of 32 (2.32 against 2.22 ms at about 1024
// blocks per layer; 2.30 and 2.36 ms at 512 and 2048 blocks).
// X rows are zero where the row of q = q0 - 1 + j plus ky - 1 leaves the
// image (or q is outside 0 .. P-1).  A tap (ky, kx) reads X[ky] from row kx
// on, so the three kx taps share one staged tile; the taps that would wrap
// across a row edge (kx = 0 at column 0, kx = 2 at column W-1) are removed
// by zeroing those pixels in the dz fragment, in registers.
//
// The matrix fragments need 8 consecutive pixels of one channel per lane, a
// column of the pixel-major tiles: each comes from two transposing LDS
// reads (ds_read_b64_tr_b16).  Within a group of 16 lanes, lane i receives
// element i % 4 of the 8-byte chunks read by lanes i/4, i/4+4, i/4+8 and
// i/4+12; so with lane s of the group reading row base + s/4 at channel
// 4 (s % 4), lane i gets channel i at rows base .. base + 3.
constexpr int kWP = 40;     // LDS row pitch in bf16: 32 channels + 8 padding
constexpr int kWgradChunk = 32;   // pixels staged per step of k_wgrad

typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
typedef __attribute__((address_space(3))) bf16x4 *lds_bf16x4_ptr;

// channels [16 h, 16 h + 16) of rows base .. base + 7 of a pixel-major LDS
// tile, as this lane's 8-pixel fragment
__device__ __forceinline__ bf16x8 tr_fragment(const bf16 *tile, int base, int h, int lane) {
    const int s = lane & 15;
    const bf16 *p0 = tile + (base + (s >> 2)) * kWP + 16 * h + 4 * (s & 3);
    const bf16 *p1 = p0 + 4 * kWP;
    const bf16x4 lo = __builtin_amdgcn_ds_read_tr16_b64_v4bf16((lds_bf16x4_ptr)(p0));
    const bf16x4 hi = __builtin_amdgcn_ds_read_tr16_b64_v4bf16((lds_bf16x4_ptr)(p1));
    return bf16x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
}

template <int CH>
__global__ __launch_bounds__(256) void k_wgrad(const bf16 *__restrict__ x,
                                               const bf16 *__restrict__ dz,
                                               float *__restrict__ part, int N, int H, int W,
                                               int Ci, int Co) {
    static_assert(CH % 32 == 0, "chunks of whole 32-pixel fragments");
    constexpr int NH = CH / 32;                   // 32-pixel halves per chunk
    constexpr int XR = CH + 2;                    // staged X rows per ky
    __shared__ __attribute__((aligned(16))) bf16 Z[CH * kWP];
    __shared__ __attribute__((aligned(16))) bf16 X[3][XR * kWP];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, t = threadIdx.x;
    const int nci = Ci / 32;
    const int cit = blockIdx.y % nci, cot = blockIdx.y / nci;
    const int64_t P = (int64_t)N * H * W;
    const int64_t nchunk = (P + CH - 1) / CH;
    const int mt = wave >> 1, nt = wave & 1;      // this wave's 16 x 16 sub-tile
    const int g = lane >> 4;                      // pixel group: rows 8 g .. 8 g + 7
    f32x4 acc[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) acc[k] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.f;                               // bias partial (ci tile 0)
    const bool do_bias = cit == 0;
    const bf16 zero = (bf16)0.f;
    // staging: CH x 4 pieces of Z, then 3 x (CH + 2) x 4 pieces of X (16
    // bytes each), kPer per thread; the pieces of the next chunk are loaded
    // into registers while the current chunk computes.  Column and image row
    // of the chunk's first pixel advance incrementally from chunk to chunk,
    // and the few divisions left are high multiplies, so the index
    // arithmetic stays small against the MFMAs.
    constexpr int kZ = CH * 4;
    constexpr int kPieces = kZ + 3 * XR * 4;
    constexpr int kPer = (kPieces + 255) / 256;
    const SmallDiv dW((unsigned)W), dH((unsigned)H);
    const int64_t step = (int64_t)gridDim.x * CH;          // pixels between a block's chunks
    const int dcol = (int)(step % W);
    const int drow = (int)((step / W) % H);
    int col0 = (int)(((int64_t)blockIdx.x * CH) % W);
    int row0 = (int)(((int64_t)blockIdx.x * CH / W) % H);
    uint4 pre[kPer];
    auto fetch = [&](int64_t q0, int c0, int r0, uint4 *out) {
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int idx = t + 256 * u;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (idx < kZ) {
                const int j = idx >> 2, c = (idx & 3) * 8;
                const int64_t q = q0 + j;
                if (q < P) v = *reinterpret_cast<const uint4 *>(dz + q * Co + cot * 32 + c);
            } else if (idx < kPieces) {
                const int r = idx - kZ;
                const int ky = r / (XR * 4), j = (r >> 2) % XR, c = (r & 3) * 8;
                const int64_t q = q0 - 1 + j;
                if (q >= 0 && q < P) {
                    const int d = c0 - 1 + j;                    // >= -1
                    const int row = r0 + (d >= 0 ? (int)dW.div((unsigned)d) : -1);
                    const int yy = (int)dH.mod((unsigned)(row + H)) + ky - 1;
                    if (yy >= 0 && yy < H)
                        v = *reinterpret_cast<const uint4 *>(
                            x + (q + (int64_t)(ky - 1) * W) * Ci + cit * 32 + c);
                }
            }
            out[u] = v;
        }
    };
    if ((int64_t)blockIdx.x < nchunk) fetch((int64_t)blockIdx.x * CH, col0, row0, pre);
    for (int64_t ch = blockIdx.x; ch < nchunk; ch += gridDim.x) {
        __syncthreads();   // previous chunk's reads done
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int idx = t + 256 * u;
            if (idx < kZ) {
                *reinterpret_cast<uint4 *>(&Z[(idx >> 2) * kWP + (idx & 3) * 8]) = pre[u];
            } else if (idx < kPieces) {
                const int r = idx - kZ;
                *reinterpret_cast<uint4 *>(&X[r / (XR * 4)][((r >> 2) % XR) * kWP + (r & 3) * 8]) =
                    pre[u];
            }
        }
        __syncthreads();
        // column and row of the next chunk's first pixel
        int ncol = col0 + dcol, nrow = row0 + drow;
        if (ncol >= W) {
            ncol -= W;
            ++nrow;
        }
        if (nrow >= H) nrow -= H;
        if (ch + gridDim.x < nchunk) fetch((ch + gridDim.x) * CH, ncol, nrow, pre);
#pragma unroll
        for (int hf = 0; hf < NH; ++hf) {
            // dz fragment (channels 16 mt .. +15, pixels 32 hf + 8 g .. +7)
            // and its two edge-masked copies
            const int pb = 32 * hf + 8 * g;
            const bf16x8 a1 = tr_fragment(Z, pb, mt, lane);
            bf16x8 a0 = a1, a2 = a1;
            int col = (int)dW.mod((unsigned)(col0 + pb));
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                if (col == 0) a0[e] = zero;
                if (col == W - 1) a2[e] = zero;
                col = col + 1 == W ? 0 : col + 1;
            }
#pragma unroll
            for (int ky = 0; ky < 3; ++ky) {
#pragma unroll
                for (int kx = 0; kx < 3; ++kx) {
                    const bf16x8 bv = tr_fragment(X[ky], pb + kx, nt, lane);
                    const bf16x8 a = kx == 0 ? a0 : (kx == 1 ? a1 : a2);
                    acc[ky * 3 + kx] = mfma(a, bv, acc[ky * 3 + kx]);
                }
            }
        }
        if (do_bias && t < 32) {
#pragma unroll 8
            for (int j = 0; j < CH; ++j) bsum += (float)Z[j * kWP + t];
        }
        col0 = ncol;
        row0 = nrow;
    }
    // this block's partial sums: record blockIdx.x of Co 9 Ci weight sums
    // followed by Co bias sums
    const size_t tile = (size_t)Co * 9 * Ci;
    float *o = part + blockIdx.x * (tile + Co);
#pragma unroll
    for (int k = 0; k < 9; ++k)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int co = cot * 32 + 16 * mt + 4 * (lane >> 4) + r;
            const int ci = cit * 32 + 16 * nt + (lane & 15);
            o[((size_t)co * 9 + k) * Ci + ci] = acc[k][r];
        }
    if (do_bias && t < 32) o[tile + cot * 32 + t] = bsum;
}

// sum_k part[k][i] over the nsplit records of n = n1 + n2 floats, written
// to out1[i] for i < n1 and to out2[i - n1] after: 64 outputs per block, GR
// groups of waves summing the splits k = g (mod GR) with four loads in
// flight each, combined in a fixed order (deterministic).  GR = 16 gives
// small layers (few outputs, many splits) more loads in flight per output.
template <int GR>
__global__ __launch_bounds__(64 * GR) void k_reduce(const float *__restrict__ part,
                                                    float *__restrict__ out1,
                                                    float *__restrict__ out2, size_t n1, size_t n,
                                                    int nsplit) {
    __shared__ float red[GR][64];
    const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
    const size_t i = (size_t)blockIdx.x * 64 + lane;
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    if (i < n) {
        int k = g;
        for (; k + 3 * GR < nsplit; k += 4 * GR) {
            s0 += part[(size_t)k * n + i];
            s1 += part[(size_t)(k + GR) * n + i];
            s2 += part[(size_t)(k + 2 * GR) * n + i];
            s3 += part[(size_t)(k + 3 * GR) * n + i];
        }
        if (k < nsplit) s0 += part[(size_t)k * n + i];
        if (k + GR < nsplit) s1 += part[(size_t)(k + GR) * n + i];
        if (k + 2 * GR < nsplit) s2 += part[(size_t)(k + 2 * GR) * n + i];
    }
    red[g][lane] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    if (g != 0 || i >= n) return;
    float tot = red[0][lane];
#pragma unroll
    for (int v = 1; v < GR; ++v) tot += red[v][lane];
    if (i < n1)
        out1[i] = tot;
    else
        out2[i - n1] = tot;
}

// ---------------------------------------------------------------------------
// Element-wise pieces.
__global__ void k_relu_bwd(const bf16 *__restrict__ y, const bf16 *__restrict__ dy,
                           bf16 *__restrict__ dz, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dz[i] = (float)y[i] > 0.f ? dy[i] : (bf16)0.f;
}

// 2x2 average pooling (H, W even) and its adjoint
__global__ void k_pool(const bf16 *__restrict__ x, bf16 *__restrict__ y, int N, int H, int W,
                       int C) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int Ho = H / 2, Wo = W / 2;
    if (i >= (size_t)N * Ho * Wo * C) return;
    const int c = (int)(i % C);
    size_t r = i / C;
    const int xo = (int)(r % Wo), yo = (int)((r / Wo) % Ho);
    const size_t n = r / ((size_t)Wo * Ho);
    const bf16 *p = x + ((n * H + 2 * yo) * W + 2 * xo) * C + c;
    const float s = (float)p[0] + (float)p[C] + (float)p[(size_t)W * C] + (float)p[(size_t)W * C + C];
    y[i] = (bf16)(0.25f * s);
}
__global__ void k_pool_bwd(const bf16 *__restrict__ dy, const bf16 *__restrict__ s,
                           bf16 *__restrict__ dx, int N, int H, int W, int C) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)N * H * W * C) return;
    const int c = (int)(i % C);
    size_t r = i / C;
    const int xx = (int)(r % W), yy = (int)((r / W) % H);
    const size_t n = r / ((size_t)W * H);
    float v = 0.25f * (float)dy[((n * (H / 2) + yy / 2) * (W / 2) + xx / 2) * C + c];
    if (s) v += (float)s[i];
    dx[i] = (bf16)v;
}

// nearest 2x upsampling plus a skip: y = up(x) + s (s may be null), and the
// adjoint of the upsampling (sum of each 2x2 block)
__global__ void k_up_add(const bf16 *__restrict__ x, const bf16 *__restrict__ s,
                         bf16 *__restrict__ y, int N, int Ho, int Wo, int C) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)N * Ho * Wo * C) return;
    const int c = (int)(i % C);
    size_t r = i / C;
    const int xx = (int)(r % Wo), yy = (int)((r / Wo) % Ho);
    const size_t n = r / ((size_t)Wo * Ho);
    float v = (float)x[((n * (Ho / 2) + yy / 2) * (Wo / 2) + xx / 2) * C + c];
    if (s) v += (float)s[i];
    y[i] = (bf16)v;
}
__global__ void k_up_bwd(const bf16 *__restrict__ dy, bf16 *__restrict__ dx, int N, int Hi,
                         int Wi, int C) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)N * Hi * Wi * C) return;
    const int c = (int)(i % C);
    size_t r = i / C;
    const int xx = (int)(r % Wi), yy = (int)((r / Wi) % Hi);
    const size_t n = r / ((size_t)Wi * Hi);
    const int W2 = 2 * Wi;
    const bf16 *p = dy + ((n * 2 * Hi + 2 * yy) * W2 + 2 * xx) * C + c;
    dx[i] = (bf16)((float)p[0] + (float)p[C] + (float)p[(size_t)W2 * C] +
                   (float)p[(size_t)W2 * C + C]);
}

__global__ void k_add(const bf16 *a, const bf16 *b,
                      bf16 *y, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = (bf16)((float)a[i] + (float)b[i]);
}

// The same element-wise kernels on 8 channels (16 bytes) per thread, used
// when the channel count is a multiple of 8 and every operand is 16-byte
// aligned; each value is computed exactly as in the one-channel kernels.
__device__ __forceinline__ bf16x8 ld8(const bf16 *p) { return *reinterpret_cast<const bf16x8 *>(p); }
__device__ __forceinline__ void st8(bf16 *p, bf16x8 v) { *reinterpret_cast<bf16x8 *>(p) = v; }

__global__ void k_relu_bwd8(const bf16 *__restrict__ y, const bf16 *__restrict__ dy,
                            bf16 *__restrict__ dz, size_t n8) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n8) return;
    const bf16x8 a = ld8(y + 8 * i), g = ld8(dy + 8 * i);
    bf16x8 o;
#pragma unroll
    for (int k = 0; k < 8; ++k) o[k] = (float)a[k] > 0.f ? g[k] : (bf16)0.f;
    st8(dz + 8 * i, o);
}

__global__ void k_add8(const bf16 *a, const bf16 *b, bf16 *y, size_t n8) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n8) return;
    const bf16x8 u = ld8(a + 8 * i), v = ld8(b + 8 * i);
    bf16x8 o;
#pragma unroll
    for (int k = 0; k < 8; ++k) o[k] = (bf16)((float)u[k] + (float)v[k]);
    st8(y + 8 * i, o);
}

__global__ void k_pool8(const bf16 *__restrict__ x, bf16 *__restrict__ y, int N, int H, int W,
                        int C) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int Ho = H / 2, Wo = W / 2, C8 = C / 8;
    if (i >= (size_t)N * Ho * Wo * C8) return;
    const int c = (int)(i % C8) * 8;
    const size_t r = i / C8;
    const int xo = (int)(r % Wo), yo = (int)((r / Wo) % Ho);
    const size_t n = r / ((size_t)Wo * Ho);
    const bf16 *p = x + ((n * H + 2 * yo) * W + 2 * xo) * C + c;
    const bf16x8 a = ld8(p), b = ld8(p + C), d = ld8(p + (size_t)W * C), e = ld8(p + (size_t)W * C + C);
    bf16x8 o;
#pragma unroll
    for (int k = 0; k < 8; ++k)
        o[k] = (bf16)(0.25f * ((float)a[k] + (float)b[k] + (float)d[k] + (float)e[k]));
    st8(y + r * C + c, o);
}

__global__ void k_pool_bwd8(const bf16 *__restrict__ dy, const bf16 *__restrict__ s,
                            bf16 *__restrict__ dx, int N, int H, int W, int C) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int C8 = C / 8;
    if (i >= (size_t)N * H * W * C8) return;
    const int c = (int)(i % C8) * 8;
    const size_t r = i / C8;
    const int xx = (int)(r % W), yy = (int)((r / W) % H);
    const size_t n = r / ((size_t)W * H);
    const bf16x8 g = ld8(dy + ((n * (H / 2) + yy / 2) * (W / 2) + xx / 2) * C + c);
    bf16x8 o;
    if (s) {
        const bf16x8 v = ld8(s + r * C + c);
#pragma unroll
        for (int k = 0; k < 8; ++k) o[k] = (bf16)(0.25f * (float)g[k] + (float)v[k]);
    } else {
#pragma unroll
        for (int k = 0; k < 8; ++k) o[k] = (bf16)(0.25f * (float)g[k]);
    }
    st8(dx + r * C + c, o);
}

__global__ void k_up_add8(const bf16 *__restrict__ x, const bf16 *__restrict__ s,
                          bf16 *__restrict__ y, int N, int Ho, int Wo, int C) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int C8 = C / 8;
    if (i >= (size_t)N * Ho * Wo * C8) return;
    const int c = (int)(i % C8) * 8;
    const size_t r = i / C8;
    const int xx = (int)(r % Wo), yy = (int)((r / Wo) % Ho);
    const size_t n = r / ((size_t)Wo * Ho);
    const bf16x8 u = ld8(x + ((n * (Ho / 2) + yy / 2) * (Wo / 2) + xx / 2) * C + c);
    bf16x8 o;
    if (s) {
        const bf16x8 v = ld8(s + r * C + c);
#pragma unroll
        for (int k = 0; k < 8; ++k) o[k] = (bf16)((float)u[k] + (float)v[k]);
    } else {
        o = u;
    }
    st8(y + r * C + c, o);
}

__global__ void k_up_bwd8(const bf16 *__restrict__ dy, bf16 *__restrict__ dx, int N, int Hi,
                          int Wi, int C) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int C8 = C / 8;
    if (i >= (size_t)N * Hi * Wi * C8) return;
    const int c = (int)(i % C8) * 8;
    const size_t r = i / C8;
    const int xx = (int)(r % Wi), yy = (int)((r / Wi) % Hi);
    const size_t n = r / ((size_t)Wi * Hi);
    const int W2 = 2 * Wi;
    const bf16 *p = dy + ((n * 2 * Hi + 2 * yy) * W2 + 2 * xx) * C + c;
    const bf16x8 a = ld8(p), b = ld8(p + C), d = ld8(p + (size_t)W2 * C),
                 e = ld8(p + (size_t)W2 * C + C);
    bf16x8 o;
#pragma unroll
    for (int k = 0; k < 8; ++k)
        o[k] = (bf16)((float)a[k] + (float)b[k] + (float)d[k] + (float)e[k]);
    st8(dx + r * C + c, o);
}

// Mean squared error over the first `cout` channels of y [P][C] against
// target [P][cout] (FP32): per-block partial sums (double) and the gradient
// dy = 2 (y - t) / (P cout) (zero in the other channels).
__global__ __launch_bounds__(256) void k_mse(const bf16 *__restrict__ y,
                                             const float *__restrict__ tgt,
                                             bf16 *__restrict__ dy, double *__restrict__ partial,
                                             size_t P, int C, int cout) {
    __shared__ double red[256];
    double acc = 0.0;
    const double scale = 2.0 / ((double)P * cout);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < P * C;
         i += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        const size_t p = i / C;
        float g = 0.f;
        if (c < cout) {
            const double d = (double)(float)y[i] - (double)tgt[p * cout + c];
            acc += d * d;
            g = (float)(scale * d);
        }
        if (dy) dy[i] = (bf16)g;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// The same loss per pixel, for C a multiple of 8 and 16-byte aligned rows:
// a thread reads the cout channels of a pixel it needs and writes the whole
// dy row as 16-byte pieces (zero past cout), with no per-element division.
__global__ __launch_bounds__(256) void k_mse_px(const bf16 *__restrict__ y,
                                                const float *__restrict__ tgt,
                                                bf16 *__restrict__ dy,
                                                double *__restrict__ partial, size_t P, int C,
                                                int cout) {
    __shared__ double red[256];
    double acc = 0.0;
    const double scale = 2.0 / ((double)P * cout);
    const int nv = C / 8;
    for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < P;
         p += (size_t)gridDim.x * blockDim.x) {
        for (int v = 0; v < nv; ++v) {
            uint4 out = make_uint4(0u, 0u, 0u, 0u);
            if (8 * v < cout) {
                unsigned short h[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int c = 8 * v + e;
                    float g = 0.f;
                    if (c < cout) {
                        const double d = (double)(float)y[p * C + c] - (double)tgt[p * cout + c];
                        acc += d * d;
                        g = (float)(scale * d);
                    }
                    const bf16 b = (bf16)g;
                    h[e] = __builtin_bit_cast(unsigned short, b);
                }
                out = make_uint4(h[0] | (unsigned)h[1] << 16, h[2] | (unsigned)h[3] << 16,
                                 h[4] | (unsigned)h[5] << 16, h[6] | (unsigned)h[7] << 16);
            }
            if (dy) *reinterpret_cast<uint4 *>(dy + p * C + 8 * v) = out;
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// *out = scale * sum of the partials: 64 strided sums, then a fixed-order
// tree (deterministic)
__global__ __launch_bounds__(64) void k_sum(const double *__restrict__ partial, int n,
                                            double scale, double *__restrict__ out) {
    __shared__ double red[64];
    double a = 0.0;
    for (int i = threadIdx.x; i < n; i += 64) a += partial[i];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int s = 32; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0] * scale;
}

// Adam on FP32 masters with a BF16 copy for the kernels (bf16 may be null).
__global__ void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, bf16 *__restrict__ wb, size_t n, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    if (wb) wb[i] = (bf16)wi;
}

__global__ void k_to_bf16(const float *__restrict__ a, bf16 *__restrict__ b, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (bf16)a[i];
}

// Network input / output conversion between float32 planes and NHWC bf16.
__global__ void k_pack4(const float *__restrict__ planes, const float *__restrict__ scale,
                        bf16 *__restrict__ x, int N, int H, int W, int C) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)N * H * W * C) return;
    const int c = (int)(i % C);
    const size_t p = i / C;               // pixel index n*H*W + y*W + x
    const size_t hw = (size_t)H * W;
    const size_t n = p / hw, q = p % hw;
    x[i] = c < 4 ? (bf16)(planes[(n * 4 + c) * hw + q] * scale[n * 4 + c]) : (bf16)0.f;
}
// The same packing per pixel for C a multiple of 8 and x 16-byte aligned:
// four scaled plane values and zero padding, written as 16-byte pieces.
__global__ void k_pack4_px(const float *__restrict__ planes, const float *__restrict__ scale,
                           bf16 *__restrict__ x, int N, int H, int W, int C) {
    const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t hw = (size_t)H * W;
    if (p >= (size_t)N * hw) return;
    const size_t n = p / hw, q = p - n * hw;
    unsigned short h[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const bf16 b = (bf16)(planes[(n * 4 + c) * hw + q] * scale[n * 4 + c]);
        h[c] = __builtin_bit_cast(unsigned short, b);
    }
    uint4 *row = reinterpret_cast<uint4 *>(x + p * C);
    row[0] = make_uint4(h[0] | (unsigned)h[1] << 16, h[2] | (unsigned)h[3] << 16, 0u, 0u);
    for (int v = 1; v < C / 8; ++v) row[v] = make_uint4(0u, 0u, 0u, 0u);
}
__global__ void k_unpack2(const bf16 *__restrict__ y, const float *__restrict__ scale,
                          float *__restrict__ out, int N, int H, int W, int C) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t hw = (size_t)H * W;
    if (i >= (size_t)N * 2 * hw) return;
    const size_t q = i % hw, nc = i / hw;
    const int c = (int)(nc % 2);
    const size_t n = nc / 2;
    out[i] = (float)y[(n * hw + q) * C + c] * scale[n * 2 + c];
}

unsigned blocks_for(size_t n) { return (unsigned)((n + 255) / 256); }

int status(hipError_t e) { return e == hipSuccess ? FWI_NN_OK : FWI_NN_EHIP; }

bool al16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

}  // namespace

extern "C" {

int fwi_nn_conv3x3(const void *x, const void *w, const float *bias, void *y, int32_t N,
                   int32_t H, int32_t W, int32_t Ci, int32_t Co, int32_t relu, void *stream) {
    if (!x || !w || !y || N < 1 || H < 1 || W < 1 || H > 32768 || W > 32768 || Ci < 32 ||
        Co < 32 || Ci % 32 || Co % 32 || !al16(x) || !al16(w))
        return FWI_NN_EINVAL;
    if ((int64_t)N * H * W >= (int64_t)1 << 36) return FWI_NN_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t P = (int64_t)N * H * W;
    const bf16 *xb = static_cast<const bf16 *>(x);
    const bf16 *wb = static_cast<const bf16 *>(w);
    bf16 *yb = static_cast<bf16 *>(y);
    // LDS-tiled kernel when it still gives the chip enough blocks, with the
    // narrower channel tile where only that one does, and 64-pixel blocks
    // where 128-pixel blocks would leave fewer than two blocks per CU
    int bn = Co % 64 == 0 ? 64 : 32;
    if (bn == 64 && (P + 127) / 128 * (Co / 64) < 256) bn = 32;
    const int64_t lds_blocks = (P + 127) / 128 * (Co / bn);
    if (lds_blocks >= 256) {
        // (the 64-pixel tile below 1024 blocks of 128 made the network's
        // 32 x 32-pixel layers slower)
        const int bm = lds_blocks < 512 ? 64 : 128;
        const dim3 grid((unsigned)((P + bm - 1) / bm), (unsigned)(Co / bn));
        if (bn == 64 && bm == 128)
            hipLaunchKernelGGL((k_conv3x3_lds<64, 128>), grid, dim3(256), 0, st, xb, wb, bias, yb,
                               N, H, W, Ci, Co, relu);
        else if (bn == 64)
            hipLaunchKernelGGL((k_conv3x3_lds<64, 64>), grid, dim3(256), 0, st, xb, wb, bias, yb,
                               N, H, W, Ci, Co, relu);
        else if (bm == 128)
            hipLaunchKernelGGL((k_conv3x3_lds<32, 128>), grid, dim3(256), 0, st, xb, wb, bias, yb,
                               N, H, W, Ci, Co, relu);
        else
            hipLaunchKernelGGL((k_conv3x3_lds<32, 64>), grid, dim3(256), 0, st, xb, wb, bias, yb,
                               N, H, W, Ci, Co, relu);
        return status(hipGetLastError());
    }
    // small layers: 64-pixel blocks of 32-channel tiles (four times the
    // blocks of the LDS tiling)
    const dim3 grid((unsigned)((P + 63) / 64), (unsigned)(Co / 32));
    hipLaunchKernelGGL((k_conv3x3<2, 1>), grid, dim3(256), 0, st, xb, wb, bias, yb, N, H, W, Ci,
                       Co, relu);
    return status(hipGetLastError());
}

int fwi_nn_flip(const void *w, void *wf, int32_t Ci, int32_t Co, void *stream) {
    if (!w || !wf || Ci < 1 || Co < 1) return FWI_NN_EINVAL;
    const size_t n = (size_t)Co * 9 * Ci;
    hipLaunchKernelGGL(k_flip, dim3(blocks_for(n)), dim3(256), 0, static_cast<hipStream_t>(stream),
                       static_cast<const bf16 *>(w), static_cast<bf16 *>(wf), Ci, Co);
    return status(hipGetLastError());
}

int fwi_nn_flip_layers(const void *w, void *wf, int32_t nlayers, const int64_t *off,
                       const int32_t *ci, const int32_t *co, void *stream) {
    if (!w || !wf || !off || !ci || !co || nlayers < 1 || nlayers > kFlipMax)
        return FWI_NN_EINVAL;
    FlipTable tb{};
    tb.n = nlayers;
    int64_t end = 0;
    for (int l = 0; l < nlayers; ++l) {
        if (off[l] < end || ci[l] < 1 || co[l] < 1 || (int64_t)9 * ci[l] * co[l] >= (1ll << 31))
            return FWI_NN_EINVAL;
        tb.off[l] = off[l];
        tb.ci[l] = ci[l];
        tb.co[l] = co[l];
        end = off[l] + (int64_t)9 * ci[l] * co[l];
    }
    hipLaunchKernelGGL(k_flip_layers, dim3(blocks_for((size_t)end)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), static_cast<const bf16 *>(w),
                       static_cast<bf16 *>(wf), tb, end);
    return status(hipGetLastError());
}

size_t fwi_nn_wgrad_workspace(int32_t Ci, int32_t Co, int32_t nsplit) {
    return ((size_t)nsplit * Co * 9 * Ci + (size_t)nsplit * Co) * sizeof(float);
}

int fwi_nn_wgrad(const void *x, const void *dz, float *dw, float *db, int32_t N, int32_t H,
                 int32_t W, int32_t Ci, int32_t Co, int32_t nsplit, void *ws, size_t ws_bytes,
                 void *stream) {
    if (!x || !dz || !dw || !db || !ws || N < 1 || H < 1 || W < 1 || H > 32768 || W > 32768 ||
        Ci < 32 || Co < 32 ||
        Ci % 32 || Co % 32 || nsplit < 1 || nsplit > 65535 || !al16(x) || !al16(dz) ||
        (int64_t)N * H * W >= (int64_t)1 << 36 ||
        ws_bytes < fwi_nn_wgrad_workspace(Ci, Co, nsplit))
        return FWI_NN_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    float *part = static_cast<float *>(ws);
    hipLaunchKernelGGL(k_wgrad<kWgradChunk>, dim3(nsplit, (Co / 32) * (Ci / 32)), dim3(256), 0, st,
                       static_cast<const bf16 *>(x), static_cast<const bf16 *>(dz), part, N, H, W,
                       Ci, Co);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return FWI_NN_EHIP;
    const size_t nw = (size_t)Co * 9 * Ci, n = nw + Co;
    const unsigned nb = (unsigned)((n + 63) / 64);
    // sixteen wave groups where the outputs give fewer than 1024 blocks
    if (nb < 1024)
        hipLaunchKernelGGL(k_reduce<16>, dim3(nb), dim3(1024), 0, st, part, dw, db, nw, n, nsplit);
    else
        hipLaunchKernelGGL(k_reduce<4>, dim3(nb), dim3(256), 0, st, part, dw, db, nw, n, nsplit);
    return status(hipGetLastError());
}

int fwi_nn_relu_bwd(const void *y, const void *dy, void *dz, size_t n, void *stream) {
    if (!y || !dy || !dz) return FWI_NN_EINVAL;
    if (n == 0) return FWI_NN_OK;
    if (n % 8 == 0 && al16(y) && al16(dy) && al16(dz))
        hipLaunchKernelGGL(k_relu_bwd8, dim3(blocks_for(n / 8)), dim3(256), 0,
                           static_cast<hipStream_t>(stream), static_cast<const bf16 *>(y),
                           static_cast<const bf16 *>(dy), static_cast<bf16 *>(dz), n / 8);
    else
        hipLaunchKernelGGL(k_relu_bwd, dim3(blocks_for(n)), dim3(256), 0,
                           static_cast<hipStream_t>(stream), static_cast<const bf16 *>(y),
                           static_cast<const bf16 *>(dy), static_cast<bf16 *>(dz), n);
    return status(hipGetLastError());
}

int fwi_nn_pool2(const void *x, void *y, int32_t N, int32_t H, int32_t W, int32_t C, void *stream) {
    if (!x || !y || N < 1 || H < 2 || W < 2 || H % 2 || W % 2 || C < 1) return FWI_NN_EINVAL;
    const size_t n = (size_t)N * (H / 2) * (W / 2) * C;
    if (C % 8 == 0 && al16(x) && al16(y))
        hipLaunchKernelGGL(k_pool8, dim3(blocks_for(n / 8)), dim3(256), 0,
                           static_cast<hipStream_t>(stream), static_cast<const bf16 *>(x),
                           static_cast<bf16 *>(y), N, H, W, C);
    else
        hipLaunchKernelGGL(k_pool, dim3(blocks_for(n)), dim3(256), 0,
                           static_cast<hipStream_t>(stream), static_cast<const bf16 *>(x),
                           static_cast<bf16 *>(y), N, H, W, C);
    return status(hipGetLastError());
}

int fwi_nn_pool2_bwd_add(const void *dy, const void *skip, void *dx, int32_t N, int32_t H,
                         int32_t W, int32_t C, void *stream) {
    if (!dy || !dx || N < 1 || H < 2 || W < 2 || H % 2 || W % 2 || C < 1) return FWI_NN_EINVAL;
    const size_t n = (size_t)N * H * W * C;
    const bf16 *sb = static_cast<const bf16 *>(skip);
    if (C % 8 == 0 && al16(dy) && al16(dx) && (!skip || al16(skip)))
        hipLaunchKernelGGL(k_pool_bwd8, dim3(blocks_for(n / 8)), dim3(256), 0,
                           static_cast<hipStream_t>(stream), static_cast<const bf16 *>(dy), sb,
                           static_cast<bf16 *>(dx), N, H, W, C);
    else
        hipLaunchKernelGGL(k_pool_bwd, dim3(blocks_for(n)), dim3(256), 0,
                           static_cast<hipStream_t>(stream), static_cast<const bf16 *>(dy), sb,
                           static_cast<bf16 *>(dx), N, H, W, C);
    return status(hipGetLastError());
}

int fwi_nn_pool2_bwd(const void *dy, void *dx, int32_t N, int32_t H, int32_t W, int32_t C,
                     void *stream) {
    return fwi_nn_pool2_bwd_add(dy, nullptr, dx, N, H, W, C, stream);
}

int fwi_nn_up2_add(const void *x, const void *skip, void *y, int32_t N, int32_t Ho, int32_t Wo,
                   int32_t C, void *stream) {
    if (!x || !y || N < 1 || Ho < 2 || Wo < 2 || Ho % 2 || Wo % 2 || C < 1) return FWI_NN_EINVAL;
    const size_t n = (size_t)N * Ho * Wo * C;
    if (C % 8 == 0 && al16(x) && al16(y) && (!skip || al16(skip)))
        hipLaunchKernelGGL(k_up_add8, dim3(blocks_for(n / 8)), dim3(256), 0,
                           static_cast<hipStream_t>(stream), static_cast<const bf16 *>(x),
                           static_cast<const bf16 *>(skip), static_cast<bf16 *>(y), N, Ho, Wo, C);
    else
        hipLaunchKernelGGL(k_up_add, dim3(blocks_for(n)), dim3(256), 0,
                           static_cast<hipStream_t>(stream), static_cast<const bf16 *>(x),
                           static_cast<const bf16 *>(skip), static_cast<bf16 *>(y), N, Ho, Wo, C);
    return status(hipGetLastError());
}

int fwi_nn_up2_bwd(const void *dy, void *dx, int32_t N, int32_t Hi, int32_t Wi, int32_t C,
                   void *stream) {
    if (!dy || !dx || N < 1 || Hi < 1 || Wi < 1 || C < 1) return FWI_NN_EINVAL;
    const size_t n = (size_t)N * Hi * Wi * C;
    if (C % 8 == 0 && al16(dy) && al16(dx))
        hipLaunchKernelGGL(k_up_bwd8, dim3(blocks_for(n / 8)), dim3(256), 0,
                           static_cast<hipStream_t>(stream), static_cast<const bf16 *>(dy),
                           static_cast<bf16 *>(dx), N, Hi, Wi, C);
    else
        hipLaunchKernelGGL(k_up_bwd, dim3(blocks_for(n)), dim3(256), 0,
                           static_cast<hipStream_t>(stream), static_cast<const bf16 *>(dy),
                           static_cast<bf16 *>(dx), N, Hi, Wi, C);
    return status(hipGetLastError());
}

int fwi_nn_add(const void *a, const void *b, void *y, size_t n, void *stream) {
    if (!a || !b || !y) return FWI_NN_EINVAL;
    if (n == 0) return FWI_NN_OK;
    if (n % 8 == 0 && al16(a) && al16(b) && al16(y))
        hipLaunchKernelGGL(k_add8, dim3(blocks_for(n / 8)), dim3(256), 0,
                           static_cast<hipStream_t>(stream), static_cast<const bf16 *>(a),
                           static_cast<const bf16 *>(b), static_cast<bf16 *>(y), n / 8);
    else
        hipLaunchKernelGGL(k_add, dim3(blocks_for(n)), dim3(256), 0,
                           static_cast<hipStream_t>(stream), static_cast<const bf16 *>(a),
                           static_cast<const bf16 *>(b), static_cast<bf16 *>(y), n);
    return status(hipGetLastError());
}

int fwi_nn_mse(const void *y, const float *target, void *dy, double *loss, double *partials,
               size_t P, int32_t C, int32_t cout, void *stream) {
    if (!y || !target || !loss || !partials || P == 0 || C < 1 || cout < 1 || cout > C)
        return FWI_NN_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (C % 8 == 0 && (!dy || al16(dy)))
        hipLaunchKernelGGL(k_mse_px, dim3(FWI_NN_MSE_BLOCKS), dim3(256), 0, st,
                           static_cast<const bf16 *>(y), target, static_cast<bf16 *>(dy), partials,
                           P, C, cout);
    else
        hipLaunchKernelGGL(k_mse, dim3(FWI_NN_MSE_BLOCKS), dim3(256), 0, st,
                           static_cast<const bf16 *>(y), target, static_cast<bf16 *>(dy), partials,
                           P, C, cout);
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(64), 0, st, partials, FWI_NN_MSE_BLOCKS,
                       1.0 / ((double)P * cout), loss);
    return status(hipGetLastError());
}

int fwi_nn_adam(float *w, const float *g, float *m, float *v, void *wb, size_t n, float lr,
                float beta1, float beta2, float eps, int32_t step, void *stream) {
    if (!w || !g || !m || !v || step < 1) return FWI_NN_EINVAL;
    if (n == 0) return FWI_NN_OK;
    const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(n)), dim3(256), 0, static_cast<hipStream_t>(stream),
                       w, g, m, v, static_cast<bf16 *>(wb), n, lr, beta1, beta2, eps, c1, c2);
    return status(hipGetLastError());
}

int fwi_nn_to_bf16(const float *a, void *b, size_t n, void *stream) {
    if (!a || !b) return FWI_NN_EINVAL;
    if (n == 0) return FWI_NN_OK;
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks_for(n)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), a, static_cast<bf16 *>(b), n);
    return status(hipGetLastError());
}

int fwi_nn_pack4(const float *planes, const float *scale, void *x, int32_t N, int32_t H,
                 int32_t W, int32_t C, void *stream) {
    if (!planes || !scale || !x || N < 1 || H < 1 || W < 1 || C < 4) return FWI_NN_EINVAL;
    const size_t n = (size_t)N * H * W * C;
    if (C % 8 == 0 && al16(x))
        hipLaunchKernelGGL(k_pack4_px, dim3(blocks_for((size_t)N * H * W)), dim3(256), 0,
                           static_cast<hipStream_t>(stream), planes, scale,
                           static_cast<bf16 *>(x), N, H, W, C);
    else
        hipLaunchKernelGGL(k_pack4, dim3(blocks_for(n)), dim3(256), 0,
                           static_cast<hipStream_t>(stream), planes, scale,
                           static_cast<bf16 *>(x), N, H, W, C);
    return status(hipGetLastError());
}

int fwi_nn_unpack2(const void *y, const float *scale, float *out, int32_t N, int32_t H,
                   int32_t W, int32_t C, void *stream) {
    if (!y || !scale || !out || N < 1 || H < 1 || W < 1 || C < 2) return FWI_NN_EINVAL;
    const size_t n = (size_t)N * 2 * H * W;
    hipLaunchKernelGGL(k_unpack2, dim3(blocks_for(n)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), static_cast<const bf16 *>(y), scale, out,
                       N, H, W, C);
    return status(hipGetLastError());
}

}  // extern "C"
