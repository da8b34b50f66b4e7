// nn_kernels.hip -- gfx950 kernels of the warm-start surrogate (include/lbm_nn.h):
// a 3 x 3 x 3 periodic convolution as an implicit GEMM on the matrix cores
// (v_mfma_f32_16x16x16_bf16: BF16 operands, FP32 accumulation), its weight
// gradient, and the element-wise pieces of training (ReLU mask, pooling,
// upsampling, loss, Adam).

#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <type_traits>

#include "../../include/lbm.h"
#include "../../include/lbm_nn.h"

namespace {

typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    return __builtin_bit_cast(uint16_t, __float2bfloat16(f));   // round to nearest even
}

__device__ __forceinline__ int wrapi(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Four consecutive bf16 values (8 bytes, 8-byte aligned) as an MFMA operand.
__device__ __forceinline__ s16x4 load4(const uint16_t *p) {
    return __builtin_bit_cast(s16x4, *reinterpret_cast<const uint2 *>(p));
}

// ---------------------------------------------------------------------------
// Forward convolution.  GEMM view: out[co][p] = sum_k A[co][k] B[k][p] with
// k = (t, ci).  A wave computes CT groups of 16 output channels x 64
// positions, as CT x 4 16 x 16 tiles: each B operand (16 input channels of 16
// positions at one tap) is loaded once and used by the CT groups, each A
// operand (the weights of one tap and 16 input channels) by the four
// position tiles; a block is four waves along positions.  Operand layout of
// the 16x16x16 instruction: lane l supplies A[l % 16][4 (l / 16) + j] and
// B[4 (l / 16) + j][l % 16] (j = 0..3) and receives D[4 (l / 16) + j][l % 16].
// Every output sums its taps and input channels in the same order whatever
// CT is.
// ---------------------------------------------------------------------------
template <bool OUT_F32, int CT>
__global__ void __launch_bounds__(256) conv3d_kernel(const uint16_t *__restrict__ x, int ldx,
                                                     const uint16_t *__restrict__ w, const float *__restrict__ bias,
                                                     void *__restrict__ y, int ldy, int relu, int nb, int D, int H,
                                                     int W, int ci, int co) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int co0 = blockIdx.y * 16 * CT;
    const int64_t P = (int64_t)nb * D * H * W;
    const int64_t pbase = (int64_t)blockIdx.x * 256 + wv * 64;
    const int col = lane & 15, kq = 4 * (lane >> 4);

    int pb[4], pz[4], py[4], px[4];
    bool valid[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const int64_t p = pbase + 16 * f + col;
        valid[f] = p < P;
        int64_t q = valid[f] ? p : 0;
        px[f] = (int)(q % W); q /= W;
        py[f] = (int)(q % H); q /= H;
        pz[f] = (int)(q % D);
        pb[f] = (int)(q / D);
    }
    f32x4 acc[CT][4];
#pragma unroll
    for (int g = 0; g < CT; ++g)
#pragma unroll
        for (int f = 0; f < 4; ++f) acc[g][f] = f32x4{0.f, 0.f, 0.f, 0.f};

    const s16x4 zero4 = {0, 0, 0, 0};
    for (int t = 0; t < 27; ++t) {
        const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
        const uint16_t *src[4];
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            const int64_t s = (((int64_t)pb[f] * D + wrapi(pz[f] + dz, D)) * H + wrapi(py[f] + dy, H)) * W +
                              wrapi(px[f] + dx, W);
            src[f] = x + s * ldx + kq;
        }
        const uint16_t *wa = w + ((int64_t)t * co + co0 + col) * ci + kq;
        for (int c0 = 0; c0 < ci; c0 += 16) {
            s16x4 b[4];
#pragma unroll
            for (int f = 0; f < 4; ++f) b[f] = valid[f] ? load4(src[f] + c0) : zero4;
#pragma unroll
            for (int g = 0; g < CT; ++g) {
                const s16x4 a = load4(wa + (int64_t)16 * g * ci + c0);
#pragma unroll
                for (int f = 0; f < 4; ++f) acc[g][f] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b[f], acc[g][f], 0, 0, 0);
            }
        }
    }
    // lane holds channels co0 + 16 g + kq + j of position pbase + 16 f + col
#pragma unroll
    for (int g = 0; g < CT; ++g) {
        const int cg = co0 + 16 * g + kq;
        float bj[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) bj[j] = bias ? bias[cg + j] : 0.f;
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            if (!valid[f]) continue;
            const int64_t p = pbase + 16 * f + col;
            float v[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                v[j] = acc[g][f][j] + bj[j];
                if (relu) v[j] = v[j] > 0.f ? v[j] : 0.f;
            }
            if constexpr (OUT_F32) {
                *reinterpret_cast<float4 *>(static_cast<float *>(y) + p * ldy + cg) = float4{v[0], v[1], v[2], v[3]};
            } else {
                const uint32_t lo = (uint32_t)f32_to_bf16(v[0]) | ((uint32_t)f32_to_bf16(v[1]) << 16);
                const uint32_t hi = (uint32_t)f32_to_bf16(v[2]) | ((uint32_t)f32_to_bf16(v[3]) << 16);
                *reinterpret_cast<uint2 *>(static_cast<uint16_t *>(y) + p * ldy + cg) = uint2{lo, hi};
            }
        }
    }
}

// The same convolution for lattices whose rows hold a multiple of 64 sites
// and whose planes a multiple of 4 rows: a block owns 64 x 4 positions of
// one plane (wave w: row w, four tiles of 16 positions) and CT groups of 16
// output channels.  Per chunk of 16 input channels it stages in LDS the
// 3 x 6 x 66 sites around its positions (periodic), and every tap reads its
// B operands from there; each output sums the chunks in order, within a
// chunk the taps in order.
constexpr int kLx = 66, kLy = 6, kLz = 3, kLvox = kLx * kLy * kLz;

template <bool OUT_F32, int CT>
__global__ void __launch_bounds__(256) conv3d_lds_kernel(const uint16_t *__restrict__ x, int ldx,
                                                         const uint16_t *__restrict__ w,
                                                         const float *__restrict__ bias, void *__restrict__ y,
                                                         int ldy, int relu, int D, int H, int W, int ci, int co) {
    __shared__ __attribute__((aligned(16))) uint16_t halo[kLvox * 16];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int co0 = blockIdx.y * 16 * CT;
    const int xt = W / 64, yt = H / 4;
    int q = blockIdx.x;
    const int x0 = (q % xt) * 64;
    q /= xt;
    const int y0 = (q % yt) * 4;
    q /= yt;
    const int z = q % D, b = q / D;
    const int col = lane & 15, kq = 4 * (lane >> 4);

    f32x4 acc[CT][4];
#pragma unroll
    for (int g = 0; g < CT; ++g)
#pragma unroll
        for (int f = 0; f < 4; ++f) acc[g][f] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int c0 = 0; c0 < ci; c0 += 16) {
        __syncthreads();   // the previous chunk's reads are done
        for (int piece = threadIdx.x; piece < 2 * kLvox; piece += 256) {
            const int v = piece >> 1, half = piece & 1;
            const int lz = v / (kLx * kLy), ly = (v / kLx) % kLy, lx = v % kLx;
            const int gz = wrapi(z + lz - 1, D), gy = wrapi(y0 + ly - 1, H), gx = wrapi(x0 + lx - 1, W);
            const int64_t site = (((int64_t)b * D + gz) * H + gy) * W + gx;
            *reinterpret_cast<uint4 *>(halo + v * 16 + 8 * half) =
                *reinterpret_cast<const uint4 *>(x + site * ldx + c0 + 8 * half);
        }
        __syncthreads();
        for (int t = 0; t < 27; ++t) {
            const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;   // offsets + 1
            s16x4 bv[4];
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                const int v = (dz * kLy + wv + dy) * kLx + 16 * f + col + dx;
                bv[f] = __builtin_bit_cast(s16x4, *reinterpret_cast<const uint2 *>(halo + v * 16 + kq));
            }
            const uint16_t *wa = w + ((int64_t)t * co + co0 + col) * ci + c0 + kq;
#pragma unroll
            for (int g = 0; g < CT; ++g) {
                const s16x4 a = load4(wa + (int64_t)16 * g * ci);
#pragma unroll
                for (int f = 0; f < 4; ++f) acc[g][f] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bv[f], acc[g][f], 0, 0, 0);
            }
        }
    }
    // lane holds channels co0 + 16 g + kq + j of position (x0 + 16 f + col, y0 + wv)
    const int64_t prow = (((int64_t)b * D + z) * H + y0 + wv) * W + x0;
#pragma unroll
    for (int g = 0; g < CT; ++g) {
        const int cg = co0 + 16 * g + kq;
        float bj[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) bj[j] = bias ? bias[cg + j] : 0.f;
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            const int64_t p = prow + 16 * f + col;
            float v[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                v[j] = acc[g][f][j] + bj[j];
                if (relu) v[j] = v[j] > 0.f ? v[j] : 0.f;
            }
            if constexpr (OUT_F32) {
                *reinterpret_cast<float4 *>(static_cast<float *>(y) + p * ldy + cg) = float4{v[0], v[1], v[2], v[3]};
            } else {
                const uint32_t lo = (uint32_t)f32_to_bf16(v[0]) | ((uint32_t)f32_to_bf16(v[1]) << 16);
                const uint32_t hi = (uint32_t)f32_to_bf16(v[2]) | ((uint32_t)f32_to_bf16(v[3]) << 16);
                *reinterpret_cast<uint2 *>(static_cast<uint16_t *>(y) + p * ldy + cg) = uint2{lo, hi};
            }
        }
    }
}

__global__ void flip_kernel(const uint16_t *w, uint16_t *wt, int ci, int co) {
    const int64_t n = 27LL * ci * co;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e % ci);
        const int o = (int)((e / ci) % co);
        const int t = (int)(e / ((int64_t)ci * co));
        wt[((int64_t)(26 - t) * ci + c) * co + o] = w[e];
    }
}

// ---------------------------------------------------------------------------
// Weight gradient.  GEMM view per tap: dW[co][ci] = sum_p A[co][p] B[p][ci]
// with A = dy^T and B = x shifted by the tap.  A wave owns one (tap, 16 co,
// 16 ci) tile and one chunk of positions and writes its partial tile to
// work[chunk]; a second kernel sums the chunks in order.
// ---------------------------------------------------------------------------
constexpr int kChunk = 4096;   // positions per partial sum

__global__ void __launch_bounds__(256) bwd_weight_kernel(const uint16_t *__restrict__ x, int ldx,
                                                         const uint16_t *__restrict__ dyv, int lddy,
                                                         float *__restrict__ work, int nb, int D, int H, int W,
                                                         int ci, int co, int ntiles) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int tile = blockIdx.y * 4 + wv;   // (t, co tile, ci tile)
    if (tile >= ntiles) return;
    const int nci = ci / 16, nco = co / 16;
    const int cit = tile % nci, cot = (tile / nci) % nco, t = tile / (nci * nco);
    const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
    const int64_t P = (int64_t)nb * D * H * W;
    const int64_t p0 = (int64_t)blockIdx.x * kChunk;
    const int64_t p1 = p0 + kChunk < P ? p0 + kChunk : P;
    const int col = lane & 15, kq = 4 * (lane >> 4);
    const int cA = cot * 16 + col, cB = cit * 16 + col;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int64_t pk = p0; pk < p1; pk += 16) {
        short av[4], bv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t p = pk + kq + j;
            if (p < p1) {
                int64_t q = p;
                const int xx = (int)(q % W); q /= W;
                const int yy = (int)(q % H); q /= H;
                const int zz = (int)(q % D);
                const int bb = (int)(q / D);
                const int64_t s = (((int64_t)bb * D + wrapi(zz + dz, D)) * H + wrapi(yy + dy, H)) * W + wrapi(xx + dx, W);
                av[j] = (short)dyv[p * lddy + cA];
                bv[j] = (short)x[s * ldx + cB];
            } else {
                av[j] = 0;
                bv[j] = 0;
            }
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(s16x4{av[0], av[1], av[2], av[3]},
                                                        s16x4{bv[0], bv[1], bv[2], bv[3]}, acc, 0, 0, 0);
    }
    // lane holds dW[co = cot 16 + kq + j][ci = cit 16 + col]
    float *out = work + (int64_t)blockIdx.x * 27 * co * ci;
#pragma unroll
    for (int j = 0; j < 4; ++j) out[((int64_t)t * co + cot * 16 + kq + j) * ci + cB] = acc[j];
}

// db partials: one per chunk and channel.
__global__ void bwd_bias_kernel(const uint16_t *dyv, int lddy, float *work, int64_t P, int co) {
    const int c = threadIdx.x;   // blockDim.x = co (<= 1024)
    const int64_t p0 = (int64_t)blockIdx.x * kChunk;
    const int64_t p1 = p0 + kChunk < P ? p0 + kChunk : P;
    float s = 0.f;
    for (int64_t p = p0; p < p1; ++p) s += bf16_to_f32(dyv[p * lddy + c]);
    work[(int64_t)blockIdx.x * co + c] = s;
}

// out[e] = sum over chunks of part[chunk][e], chunks in order.
__global__ void sum_chunks_kernel(const float *part, int nchunks, int64_t n, float *out) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int k = 0; k < nchunks; ++k) s += part[(int64_t)k * n + e];
        out[e] = s;
    }
}

// ---------------------------------------------------------------------------
// Element-wise pieces.
// ---------------------------------------------------------------------------
__global__ void relu_bwd_cast_kernel(const float *dy, int lddy, const uint16_t *yv, int ldy, uint16_t *out, int ldo,
                                     int64_t P, int c, int relu) {
    const int64_t n = P * c;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = e / c;
        const int k = (int)(e % c);
        float g = dy[p * lddy + k];
        if (relu && !(bf16_to_f32(yv[p * ldy + k]) > 0.f)) g = 0.f;
        out[p * ldo + k] = f32_to_bf16(g);
    }
}

// Coarse position pc of (b, z, y, x) at half resolution; fine index of child (i, j, k).
__device__ __forceinline__ int64_t child(int64_t pc, int d2, int h2, int w2, int i, int j, int k) {
    int64_t q = pc;
    const int x = (int)(q % w2); q /= w2;
    const int y = (int)(q % h2); q /= h2;
    const int z = (int)(q % d2);
    const int b = (int)(q / d2);
    return (((int64_t)b * 2 * d2 + 2 * z + i) * 2 * h2 + 2 * y + j) * 2 * w2 + 2 * x + k;
}

__global__ void pool2_fwd_kernel(const uint16_t *x, int ldx, uint16_t *y, int ldy, int64_t Pc, int d2, int h2, int w2,
                                 int c) {
    const int64_t n = Pc * c;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t pc = e / c;
        const int k = (int)(e % c);
        float s = 0.f;
        for (int q = 0; q < 8; ++q) s += bf16_to_f32(x[child(pc, d2, h2, w2, q >> 2, (q >> 1) & 1, q & 1) * ldx + k]);
        y[pc * ldy + k] = f32_to_bf16(0.125f * s);
    }
}

__global__ void pool2_bwd_kernel(const float *dy, int lddy, float *dx, int lddx, int accumulate, int64_t Pc, int d2,
                                 int h2, int w2, int c) {
    const int64_t n = Pc * c;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t pc = e / c;
        const int k = (int)(e % c);
        const float g = 0.125f * dy[pc * lddy + k];
        for (int q = 0; q < 8; ++q) {
            float *o = dx + child(pc, d2, h2, w2, q >> 2, (q >> 1) & 1, q & 1) * lddx + k;
            *o = accumulate ? *o + g : g;
        }
    }
}

__global__ void up2_fwd_kernel(const uint16_t *x, int ldx, uint16_t *y, int ldy, int64_t Pc, int d, int h, int w, int c) {
    const int64_t n = Pc * c;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t pc = e / c;
        const int k = (int)(e % c);
        const uint16_t v = x[pc * ldx + k];
        for (int q = 0; q < 8; ++q) y[child(pc, d, h, w, q >> 2, (q >> 1) & 1, q & 1) * ldy + k] = v;
    }
}

__global__ void up2_bwd_kernel(const float *dy, int lddy, float *dx, int lddx, int64_t Pc, int d, int h, int w, int c) {
    const int64_t n = Pc * c;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t pc = e / c;
        const int k = (int)(e % c);
        float s = 0.f;
        for (int q = 0; q < 8; ++q) s += dy[child(pc, d, h, w, q >> 2, (q >> 1) & 1, q & 1) * lddy + k];
        dx[pc * lddx + k] = s;
    }
}

// Loss partial sums per block (FP64), then one block sums them in order.
__global__ void mse_kernel(const float *pred, int ldp, const float *target, int ldt, const float *cw, float *dpred,
                           int lddp, double *part, int64_t P, int c) {
    __shared__ double sh[256];
    const int64_t n = P * c;
    const float inv = 1.0f / (float)P;
    double s = 0.0;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = e / c;
        const int k = (int)(e % c);
        const float r = pred[p * ldp + k] - target[p * ldt + k];
        dpred[p * lddp + k] = 2.0f * cw[k] * r * inv;
        s += (double)cw[k] * (double)r * (double)r;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void mse_final_kernel(const double *part, int nparts, int64_t P, double *loss) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int k = 0; k < nparts; ++k) s += part[k];
        *loss = s / (double)P;
    }
}

__global__ void adam_kernel(float *param, const float *grad, float *m, float *v, uint16_t *pb, int64_t n, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const float g = grad[e];
        const float mm = b1 * m[e] + (1.f - b1) * g;
        const float vv = b2 * v[e] + (1.f - b2) * g * g;
        m[e] = mm;
        v[e] = vv;
        const float p = param[e] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
        param[e] = p;
        if (pb) pb[e] = f32_to_bf16(p);
    }
}

__global__ void to_bf16_kernel(const float *x, uint16_t *y, int64_t n) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        y[e] = f32_to_bf16(x[e]);
}

// ---------------------------------------------------------------------------
// Input features and output decoding of the surrogate, on the device.
// ---------------------------------------------------------------------------
// Squared distance along one axis to the nearest solid site within +-R
// (periodic; infinity if none): pass 0 of the separable distance transform.
__global__ void dist_pass_x(const uint8_t *solid, float *g2, int D, int H, int W, int R) {
    const int64_t n = (int64_t)D * H * W;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(e % W);
        const int64_t row = e - x;
        float best = __builtin_inff();
        for (int dx = -R; dx <= R; ++dx) {
            int xx = (x + dx) % W;
            if (xx < 0) xx += W;
            if (solid[row + xx]) best = fminf(best, (float)(dx * dx));
        }
        g2[e] = best;
    }
}

// Passes 1 and 2: out(p) = min over |k| <= R of in(p + k e_axis) + k^2
// (axis 1 = y, stride W; axis 2 = z, stride H W); the last pass takes the
// square root, clipped at R sqrt(3).
__global__ void dist_pass_yz(const float *in, float *out, int D, int H, int W, int R, int axis, int last) {
    const int64_t n = (int64_t)D * H * W;
    const int L = axis == 1 ? H : D;
    const int64_t stride = axis == 1 ? (int64_t)W : (int64_t)H * W;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int c = axis == 1 ? (int)((e / W) % H) : (int)(e / ((int64_t)H * W));
        const int64_t base = e - (int64_t)c * stride;
        float best = __builtin_inff();
        for (int k = -R; k <= R; ++k) {
            int cc = (c + k) % L;
            if (cc < 0) cc += L;
            best = fminf(best, in[base + (int64_t)cc * stride] + (float)(k * k));
        }
        out[e] = last ? fminf(sqrtf(best), (float)R * 1.7320508f) : best;
    }
}

// bf16 input channels [solid, phi_A, dist / dist_scale, 0 ...] (c channels
// at stride ldx), phi_A = rho_A / (rho_A + rho_B) on fluid sites, else 0.
__global__ void features_kernel(const uint8_t *solid, const double *ra, const double *rb, const float *dist,
                                float inv_scale, uint16_t *x, int ldx, int c, int64_t n) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const bool s = solid[e] != 0;
        const double tot = ra[e] + rb[e];
        const float phi = (!s && tot > 0) ? (float)(ra[e] / tot) : 0.f;
        uint16_t *o = x + e * ldx;
        o[0] = f32_to_bf16(s ? 1.f : 0.f);
        o[1] = f32_to_bf16(phi);
        o[2] = f32_to_bf16(dist[e] * inv_scale);
        for (int k = 3; k < c; ++k) o[k] = 0;
    }
}

// Fields from the output channels [ux, uy, uz, d rho_A, d rho_B] at fluid
// sites: u = out * u_scale * g / nu_mix (nu_mix of the initial fraction,
// Eqs. 5-6), rho = max(rho0 + rho_scale * out, floor); zero on solid sites.
// Per-block FP64 sums of [rho_A0, rho_B0, rho_A, rho_B] over fluid sites go
// to part (4 per block).
__global__ void decode_kernel(const float *out, int ldo, const uint8_t *solid, const double *ra0, const double *rb0,
                              double nu_a, double nu_b, double g, float u_scale, float rho_scale, double floor,
                              double *u, double *ra, double *rb, double *part, int64_t n) {
    __shared__ double sh[4][256];
    double acc[4] = {0, 0, 0, 0};
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const float *o = out + e * ldo;
        double ux = 0, uy = 0, uz = 0, a = 0, b = 0;
        if (!solid[e]) {
            const double tot = ra0[e] + rb0[e];
            const double phi = tot > 0 ? ra0[e] / tot : 0.0;
            const double m = g / (phi * nu_a + (1.0 - phi) * nu_b);
            ux = (double)o[0] * (double)u_scale * m;
            uy = (double)o[1] * (double)u_scale * m;
            uz = (double)o[2] * (double)u_scale * m;
            a = fmax(ra0[e] + (double)rho_scale * (double)o[3], floor);
            b = fmax(rb0[e] + (double)rho_scale * (double)o[4], floor);
            acc[0] += ra0[e];
            acc[1] += rb0[e];
            acc[2] += a;
            acc[3] += b;
        }
        u[e] = ux;
        u[n + e] = uy;
        u[2 * n + e] = uz;
        ra[e] = a;
        rb[e] = b;
    }
    for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 4) part[blockIdx.x * 4 + threadIdx.x] = sh[threadIdx.x][0];
}

// Rescales rho_A, rho_B so that their fluid sums equal those of rho_A0,
// rho_B0 (the partial sums of decode_kernel, added in block order).
__global__ void rescale_kernel(const double *part, int nparts, double *ra, double *rb, int64_t n) {
    __shared__ double tot[4];
    if (threadIdx.x < 4) {
        double s = 0.0;
        for (int q = 0; q < nparts; ++q) s += part[q * 4 + threadIdx.x];
        tot[threadIdx.x] = s;
    }
    __syncthreads();
    const double fa = tot[2] > 0 ? tot[0] / tot[2] : 0.0, fb = tot[3] > 0 ? tot[1] / tot[3] : 0.0;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        ra[e] *= fa;
        rb[e] *= fb;
    }
}

constexpr int kDecodeBlocks = 1024;

int grid_for(int64_t n) {
    const int64_t b = (n + 255) / 256;
    return (int)(b < 16384 ? (b > 0 ? b : 1) : 16384);
}

int done() { return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EDEVICE; }

bool aligned8(const void *p) { return ((uintptr_t)p & 7) == 0; }

int64_t positions(int nb, int d, int h, int w) { return (int64_t)nb * d * h * w; }

bool dims_ok(int nb, int d, int h, int w) { return nb > 0 && d > 0 && h > 0 && w > 0; }

}  // namespace

extern "C" {

int nn_conv3d_fwd(const uint16_t *x, int32_t ldx, const uint16_t *w, const float *bias, void *y, int32_t ldy,
                  int32_t y_fp32, int32_t relu, int32_t nb, int32_t d, int32_t h, int32_t w_, int32_t ci, int32_t co,
                  void *stream) {
    if (!x || !w || !y || !dims_ok(nb, d, h, w_) || ci <= 0 || co <= 0 || ci % 16 || co % 16 || ldx < ci ||
        ldy < co || ldx % 4 || ldy % 4 || !aligned8(x) || !aligned8(w) || (y_fp32 ? ((uintptr_t)y & 15) : !aligned8(y)))
        return LBM_EINVAL;
    const int64_t P = positions(nb, d, h, w_);
    hipStream_t s = static_cast<hipStream_t>(stream);
    // CT groups of 16 output channels per wave: the largest of 6, 4, 3, 2, 1
    // that divides co / 16.
    const int groups = co / 16;
    const int ct = groups % 6 == 0 ? 6 : groups % 4 == 0 ? 4 : groups % 3 == 0 ? 3 : groups % 2 == 0 ? 2 : 1;
    const dim3 grid((unsigned)((P + 255) / 256), (unsigned)(groups / ct));
    // rows of a multiple of 64 sites, planes of a multiple of 4 rows, and
    // 16-byte aligned input rows: the LDS-staged form
    const bool staged = w_ % 64 == 0 && h % 4 == 0 && ldx % 8 == 0 && ((uintptr_t)x & 15) == 0;
    const dim3 sgrid((unsigned)((int64_t)nb * d * (h / 4) * (w_ / 64)), (unsigned)(groups / ct));
    auto launch = [&](auto out_f32, auto ctc) {
        if (staged)
            hipLaunchKernelGGL((conv3d_lds_kernel<decltype(out_f32)::value, decltype(ctc)::value>), sgrid, dim3(256), 0,
                               s, x, ldx, w, bias, y, ldy, relu, d, h, w_, ci, co);
        else
            hipLaunchKernelGGL((conv3d_kernel<decltype(out_f32)::value, decltype(ctc)::value>), grid, dim3(256), 0, s,
                               x, ldx, w, bias, y, ldy, relu, nb, d, h, w_, ci, co);
    };
    auto by_ct = [&](auto out_f32) {
        switch (ct) {
        case 6: launch(out_f32, std::integral_constant<int, 6>{}); break;
        case 4: launch(out_f32, std::integral_constant<int, 4>{}); break;
        case 3: launch(out_f32, std::integral_constant<int, 3>{}); break;
        case 2: launch(out_f32, std::integral_constant<int, 2>{}); break;
        default: launch(out_f32, std::integral_constant<int, 1>{}); break;
        }
    };
    if (y_fp32) by_ct(std::true_type{});
    else by_ct(std::false_type{});
    return done();
}

int nn_weights_flip(const uint16_t *w, uint16_t *wt, int32_t ci, int32_t co, void *stream) {
    if (!w || !wt || ci <= 0 || co <= 0) return LBM_EINVAL;
    hipLaunchKernelGGL(flip_kernel, dim3(grid_for(27LL * ci * co)), dim3(256), 0, static_cast<hipStream_t>(stream), w,
                       wt, ci, co);
    return done();
}

int64_t nn_bwd_weight_work(int32_t nb, int32_t d, int32_t h, int32_t w_, int32_t ci, int32_t co) {
    if (!dims_ok(nb, d, h, w_) || ci <= 0 || co <= 0) return -1;
    const int64_t nch = (positions(nb, d, h, w_) + kChunk - 1) / kChunk;
    return nch * 27 * (int64_t)co * ci;   // the bias partials (nch x co) fit in the same space
}

int nn_conv3d_bwd_weight(const uint16_t *x, int32_t ldx, const uint16_t *dy, int32_t lddy, float *dw, float *db,
                         float *work, int64_t work_floats, int32_t nb, int32_t d, int32_t h, int32_t w_, int32_t ci,
                         int32_t co, void *stream) {
    if (!x || !dy || !dw || !db || !work || !dims_ok(nb, d, h, w_) || ci <= 0 || co <= 0 || ci % 16 || co % 16 ||
        co > 1024 || ldx < ci || lddy < co)
        return LBM_EINVAL;
    if (work_floats < nn_bwd_weight_work(nb, d, h, w_, ci, co)) return LBM_EINVAL;
    const int64_t P = positions(nb, d, h, w_);
    const int nch = (int)((P + kChunk - 1) / kChunk);
    const int ntiles = 27 * (co / 16) * (ci / 16);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(bwd_weight_kernel, dim3(nch, (ntiles + 3) / 4), dim3(256), 0, s, x, ldx, dy, lddy, work, nb, d,
                       h, w_, ci, co, ntiles);
    const int64_t n = 27LL * co * ci;
    hipLaunchKernelGGL(sum_chunks_kernel, dim3(grid_for(n)), dim3(256), 0, s, work, nch, n, dw);
    hipLaunchKernelGGL(bwd_bias_kernel, dim3(nch), dim3(co), 0, s, dy, lddy, work, P, co);
    hipLaunchKernelGGL(sum_chunks_kernel, dim3(grid_for(co)), dim3(256), 0, s, work, nch, (int64_t)co, db);
    return done();
}

int nn_relu_bwd_cast(const float *dy, int32_t lddy, const uint16_t *y, int32_t ldy, uint16_t *out, int32_t ldo,
                     int64_t p, int32_t c, int32_t relu, void *stream) {
    if (!dy || !out || (relu && !y) || p <= 0 || c <= 0) return LBM_EINVAL;
    hipLaunchKernelGGL(relu_bwd_cast_kernel, dim3(grid_for(p * c)), dim3(256), 0, static_cast<hipStream_t>(stream), dy,
                       lddy, y, ldy, out, ldo, p, c, relu);
    return done();
}

int nn_pool2_fwd(const uint16_t *x, int32_t ldx, uint16_t *y, int32_t ldy, int32_t nb, int32_t d, int32_t h,
                 int32_t w_, int32_t c, void *stream) {
    if (!x || !y || !dims_ok(nb, d, h, w_) || d % 2 || h % 2 || w_ % 2 || c <= 0) return LBM_EINVAL;
    const int64_t Pc = positions(nb, d / 2, h / 2, w_ / 2);
    hipLaunchKernelGGL(pool2_fwd_kernel, dim3(grid_for(Pc * c)), dim3(256), 0, static_cast<hipStream_t>(stream), x, ldx,
                       y, ldy, Pc, d / 2, h / 2, w_ / 2, c);
    return done();
}

int nn_pool2_bwd(const float *dy, int32_t lddy, float *dx, int32_t lddx, int32_t accumulate, int32_t nb, int32_t d,
                 int32_t h, int32_t w_, int32_t c, void *stream) {
    if (!dy || !dx || !dims_ok(nb, d, h, w_) || d % 2 || h % 2 || w_ % 2 || c <= 0) return LBM_EINVAL;
    const int64_t Pc = positions(nb, d / 2, h / 2, w_ / 2);
    hipLaunchKernelGGL(pool2_bwd_kernel, dim3(grid_for(Pc * c)), dim3(256), 0, static_cast<hipStream_t>(stream), dy,
                       lddy, dx, lddx, accumulate, Pc, d / 2, h / 2, w_ / 2, c);
    return done();
}

int nn_up2_fwd(const uint16_t *x, int32_t ldx, uint16_t *y, int32_t ldy, int32_t nb, int32_t d, int32_t h, int32_t w_,
               int32_t c, void *stream) {
    if (!x || !y || !dims_ok(nb, d, h, w_) || c <= 0) return LBM_EINVAL;
    const int64_t Pc = positions(nb, d, h, w_);
    hipLaunchKernelGGL(up2_fwd_kernel, dim3(grid_for(Pc * c)), dim3(256), 0, static_cast<hipStream_t>(stream), x, ldx, y,
                       ldy, Pc, d, h, w_, c);
    return done();
}

int nn_up2_bwd(const float *dy, int32_t lddy, float *dx, int32_t lddx, int32_t nb, int32_t d, int32_t h, int32_t w_,
               int32_t c, void *stream) {
    if (!dy || !dx || !dims_ok(nb, d, h, w_) || c <= 0) return LBM_EINVAL;
    const int64_t Pc = positions(nb, d, h, w_);
    hipLaunchKernelGGL(up2_bwd_kernel, dim3(grid_for(Pc * c)), dim3(256), 0, static_cast<hipStream_t>(stream), dy, lddy,
                       dx, lddx, Pc, d, h, w_, c);
    return done();
}

int nn_mse(const float *pred, int32_t ldp, const float *target, int32_t ldt, const float *cw, float *dpred,
           int32_t lddp, double *loss, int64_t p, int32_t c, void *stream) {
    if (!pred || !target || !cw || !dpred || !loss || p <= 0 || c <= 0) return LBM_EINVAL;
    // the partial sums go to the loss slot's neighbours: loss[1 .. 256]
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(mse_kernel, dim3(256), dim3(256), 0, s, pred, ldp, target, ldt, cw, dpred, lddp, loss + 1, p, c);
    hipLaunchKernelGGL(mse_final_kernel, dim3(1), dim3(64), 0, s, loss + 1, 256, p, loss);
    return done();
}

int nn_adam(float *param, const float *grad, float *m, float *v, uint16_t *param_bf16, int64_t n, float lr, float b1,
            float b2, float eps, int32_t t, void *stream) {
    if (!param || !grad || !m || !v || n <= 0 || t < 1) return LBM_EINVAL;
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    hipLaunchKernelGGL(adam_kernel, dim3(grid_for(n)), dim3(256), 0, static_cast<hipStream_t>(stream), param, grad, m, v,
                       param_bf16, n, lr, b1, b2, eps, c1, c2);
    return done();
}

int nn_solid_distance(const uint8_t *solid, float *work, float *dist, int32_t d, int32_t h, int32_t w_, int32_t radius,
                      void *stream) {
    if (!solid || !work || !dist || !dims_ok(1, d, h, w_) || radius < 1) return LBM_EINVAL;
    const int64_t n = positions(1, d, h, w_);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int g = grid_for(n);
    hipLaunchKernelGGL(dist_pass_x, dim3(g), dim3(256), 0, s, solid, work, d, h, w_, radius);
    hipLaunchKernelGGL(dist_pass_yz, dim3(g), dim3(256), 0, s, work, work + n, d, h, w_, radius, 1, 0);
    hipLaunchKernelGGL(dist_pass_yz, dim3(g), dim3(256), 0, s, work + n, dist, d, h, w_, radius, 2, 1);
    return done();
}

int nn_features(const uint8_t *solid, const double *rho_a, const double *rho_b, const float *dist, float dist_scale,
                uint16_t *x, int32_t ldx, int32_t c, int64_t p, void *stream) {
    if (!solid || !rho_a || !rho_b || !dist || !x || c < 3 || ldx < c || p <= 0 || !(dist_scale > 0))
        return LBM_EINVAL;
    hipLaunchKernelGGL(features_kernel, dim3(grid_for(p)), dim3(256), 0, static_cast<hipStream_t>(stream), solid, rho_a,
                       rho_b, dist, 1.0f / dist_scale, x, ldx, c, p);
    return done();
}

int nn_decode_fields(const float *out, int32_t ldo, const uint8_t *solid, const double *rho_a0, const double *rho_b0,
                     double nu_a, double nu_b, double g, float u_scale, float rho_scale, double floor, double *u,
                     double *rho_a, double *rho_b, double *work, int64_t p, void *stream) {
    if (!out || !solid || !rho_a0 || !rho_b0 || !u || !rho_a || !rho_b || !work || ldo < 5 || p <= 0 ||
        !(nu_a > 0) || !(nu_b > 0) || !(floor >= 0))
        return LBM_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(decode_kernel, dim3(kDecodeBlocks), dim3(256), 0, s, out, ldo, solid, rho_a0, rho_b0, nu_a, nu_b,
                       g, u_scale, rho_scale, floor, u, rho_a, rho_b, work, p);
    hipLaunchKernelGGL(rescale_kernel, dim3(grid_for(p)), dim3(256), 0, s, work, kDecodeBlocks, rho_a, rho_b, p);
    return done();
}

int nn_to_bf16(const float *x, uint16_t *y, int64_t n, void *stream) {
    if (!x || !y || n <= 0) return LBM_EINVAL;
    hipLaunchKernelGGL(to_bf16_kernel, dim3(grid_for(n)), dim3(256), 0, static_cast<hipStream_t>(stream), x, y, n);
    return done();
}

}  // extern "C"
