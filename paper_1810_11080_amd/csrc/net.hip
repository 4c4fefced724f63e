// Learned source-iteration correction: a small 3D U-Net over the element
// grid (BF16 convolution weights, FP32 activations and accumulation, FP32
// master weights with Adam), its training kernels, and the kernels that turn
// a sweep's scalar-flux residual into network input and apply the network's
// correction (FP64).  The convolutions (forward, data gradient, weight
// gradient) run on the matrix cores as implicit GEMMs in BF16 MFMA tiles
// with FP32 accumulation; FP32 activations and gradients enter them as pairs
// of BF16 terms.
//
// Network (widths c0, c1, c2; 3x3x3 convolutions, zero padding 1, bias,
// leaky ReLU slope 0.1 except on the output layer):
//   L0: e0a 3->c0, e0b c0->c0                       (e0b output = skip s0)
//   L1: e1a c0->c1 stride 2, e1b c1->c1             (e1b output = skip s1)
//   L2: e2a c1->c2 stride 2, e2b, e2c c2->c2
//   u1a c2->c1 at L2, nearest x2 upsample (cropped) + s1, u1b c1->c1
//   u0a c1->c0 at L1, nearest x2 upsample (cropped) + s0, u0b c0->c0
//   out c0->1
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "device.hpp"
#include "net.hpp"

namespace snsw {

namespace {

constexpr float kSlope = 0.1f;

// float -> bfloat16, round to nearest even; NaN stays a quiet NaN
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (uint16_t)((u >> 16) | 0x0040u);
    const uint32_t bias = 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)((u + bias) >> 16);
}

__host__ __device__ inline int out_size(int n, int s) { return (n - 1) / s + 1; }


// g *= act'(y) for the leaky ReLU (y has the sign of its input)
__global__ void act_backward_kernel(const float* __restrict__ y, float* __restrict__ g, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n && !(y[t] > 0.0f)) g[t] *= kSlope;
}

// h = upsample2(low) cropped to (Z, Y, X), plus skip
__global__ void upsample_add_kernel(const float* __restrict__ low, const float* __restrict__ skip,
                                    float* __restrict__ h, int BC, int Z, int Y, int X, int z, int y, int x) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nv = (int64_t)Z * Y * X;
    if (t >= BC * nv) return;
    const int64_t bc = t / nv;
    const int v = (int)(t - bc * nv);
    const int xx = v % X, yy = (v / X) % Y, zz = v / (X * Y);
    h[t] = low[((bc * z + zz / 2) * y + yy / 2) * x + xx / 2] + skip[t];
}

// g_low[bc][v] = sum of g_h over the (up to 8) fine cells v maps to
__global__ void upsample_back_kernel(const float* __restrict__ gh, float* __restrict__ glow, int BC, int Z, int Y,
                                     int X, int z, int y, int x) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nv = (int64_t)z * y * x;
    if (t >= BC * nv) return;
    const int64_t bc = t / nv;
    const int v = (int)(t - bc * nv);
    const int xl = v % x, yl = (v / x) % y, zl = v / (x * y);
    float acc = 0.0f;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                const int zz = 2 * zl + dz, yy = 2 * yl + dy, xx = 2 * xl + dx;
                if (zz < Z && yy < Y && xx < X) acc += gh[((bc * Z + zz) * Y + yy) * X + xx];
            }
    glow[t] = acc;
}

// Mean squared error in two deterministic passes: each block writes the sum
// of (y - t)^2 over its grid-strided share (FP64) and dy = 2 (y - t) / n;
// then one block adds the partial sums in block order: loss = sum / n.
constexpr int kMseBlocks = 256;

__global__ void __launch_bounds__(256) mse_partial_kernel(const float* __restrict__ y, const float* __restrict__ tgt,
                                                         int64_t n, float* __restrict__ dy,
                                                         double* __restrict__ partial) {
    __shared__ double red[4];
    double acc = 0.0;
    const float scale = 2.0f / (float)n;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const float d = y[t] - tgt[t];
        acc += (double)d * (double)d;
        dy[t] = scale * d;
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void mse_final_kernel(const double* __restrict__ partial, int count, int64_t n, double* __restrict__ loss) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int k = 0; k < count; ++k) s += partial[k];
    *loss = s / (double)n;
}

// Adam (bias-corrected) on the FP32 masters; refreshes the BF16 copy
__global__ void adam_kernel(float* __restrict__ theta, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, uint16_t* __restrict__ wbf, int64_t n, float lr, float b1,
                            float b2, float eps, float c1, float c2) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const float gt = g[t];
    const float mt = b1 * m[t] + (1.0f - b1) * gt;
    const float vt = b2 * v[t] + (1.0f - b2) * gt * gt;
    m[t] = mt;
    v[t] = vt;
    const float th = theta[t] - lr * (mt / c1) / (sqrtf(vt / c2) + eps);
    theta[t] = th;
    wbf[t] = f32_to_bf16(th);
}

__global__ void to_bf16_kernel(const float* __restrict__ theta, uint16_t* __restrict__ wbf, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) wbf[t] = f32_to_bf16(theta[t]);
}

// ---- scalar-flux side (FP64) ----

// avg[e] = (1^T M_e (a_e - b_e)) / (1^T M_e 1); M column-major at geo[e][0]
__global__ void elem_avg_kernel(const double* __restrict__ geo, int dim, int n, int64_t E,
                                const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ avg,
                                unsigned long long* __restrict__ maxbits) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double r = 0.0;
    if (e < E) {
        const double* M = geo + (size_t)e * (dim + 1) * n * n;
        double num = 0.0, den = 0.0;
        for (int j = 0; j < n; ++j) {
            double colsum = 0.0;
            for (int i = 0; i < n; ++i) colsum += M[(size_t)j * n + i];
            const double dj = a[e * n + j] - (b ? b[e * n + j] : 0.0);
            num += colsum * dj;
            den += colsum;
        }
        r = num / den;
        avg[e] = r;
    }
    if (maxbits) {
        double m = fabs(r);
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_xor(m, off);
            m = (o > m || o != o) ? o : m;
        }
        if ((threadIdx.x & 63) == 0) atomicMax(maxbits, (unsigned long long)__double_as_longlong(m));
    }
}

// x[0][e] = avg[e]/s, x[1][e] = log(sigma_t)/5, x[2][e] = sigma_s/sigma_t (s from maxbits; 0 if s == 0)
__global__ void net_input_kernel(const double* __restrict__ avg, const unsigned long long* __restrict__ maxbits,
                                 const double* __restrict__ sigma_t, const double* __restrict__ sigma_s, int64_t E,
                                 float* __restrict__ x) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    const double s = __longlong_as_double((long long)*maxbits);
    x[e] = s > 0.0 ? (float)(avg[e] / s) : 0.0f;
    x[E + e] = (float)(log(sigma_t[e]) / 5.0);
    x[2 * E + e] = (float)(sigma_s[e] / sigma_t[e]);
}

// t[e] = avg[e] / s
__global__ void net_target_kernel(const double* __restrict__ avg, const unsigned long long* __restrict__ maxbits,
                                  int64_t E, float* __restrict__ t) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    const double s = __longlong_as_double((long long)*maxbits);
    t[e] = s > 0.0 ? (float)(avg[e] / s) : 0.0f;
}

// phi[e][i] += s * y[e]
__global__ void apply_correction_kernel(double* __restrict__ phi, const float* __restrict__ y,
                                        const unsigned long long* __restrict__ maxbits, int n, int64_t E) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= E * n) return;
    const double s = __longlong_as_double((long long)*maxbits);
    phi[t] += s * (double)y[t / n];
}

// ---- convolutions on the matrix cores (BF16 MFMA, FP32 accumulation) ----
//
// A 3x3x3 convolution is an implicit GEMM: out[o][v] = sum_kk W[o][kk] X[kk][v]
// with kk = tap * C8 + c (tap = 9 kz + 3 ky + kx, c the input channel, C8 the
// channel count rounded up to 8 so that the eight K values a lane holds are
// eight channels of one tap).  v_mfma_f32_16x16x32_bf16 takes a 16 x 32 tile
// of W (lane l: row l mod 16, K values 8 (l / 16) .. + 7) and a 32 x 16 tile
// of X (lane l: column = voxel l mod 16, the same K values) and accumulates a
// 16 x 16 FP32 tile (lane l: rows 4 (l / 16) .. + 3, column l mod 16).  The
// weights are exact BF16 (the network's weights); an FP32 activation x is
// split into two BF16 terms, x = hi + lo up to 2^-16 relative, and both are
// multiplied, so the products keep the FP32 activations' precision.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// x = hi + lo with hi = bf16(x), lo = bf16(x - hi) (hardware conversions)
__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
    hi = (__bf16)x;
    lo = (__bf16)(x - (float)hi);
}

// Packed BF16 weights of one layer for the implicit GEMM: rows (output
// channels of the GEMM, padded to 16) of KP = 32 * ceil(27 * C8 / 32) values,
// kk = tap * C8 + c, zeros in the padding.  transposed = 0: the forward
// convolution, row o, c = input channel, W[o][c][tap].  transposed = 1: the
// data gradient, row i (input channel), c = output channel o, the tap
// mirrored: W[o][i][26 - tap].
__global__ void pack_weights_kernel(const float* __restrict__ theta, uint16_t* __restrict__ dst, int Cout, int Cin,
                                    int rows, int KP, int C8, int transposed) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)rows * KP) return;
    const int r = (int)(t / KP), kk = (int)(t - (int64_t)r * KP);
    const int tap = kk / C8, c = kk - tap * C8;
    float w = 0.0f;
    if (tap < 27) {
        if (!transposed) {
            if (r < Cout && c < Cin) w = theta[((size_t)r * Cin + c) * 27 + tap];
        } else {
            if (r < Cin && c < Cout) w = theta[((size_t)c * Cin + r) * 27 + (26 - tap)];
        }
    }
    dst[t] = f32_to_bf16(w);
}

// out[b][o][v] (+)= act(bias[o] + sum_kk W[o][kk] X[kk][v]), one wavefront per
// 16 output voxels, MT tiles of 16 output channels.  Gather of X for output
// voxel (zo, yo, xo) and tap (kz, ky, kx):
//   DILATE = false: input (s zo + kz - 1, ...) (convolution with stride s;
//                   also the data gradient of a stride-1 convolution);
//   DILATE = true:  p = zo + kz - 1 must be even, input p / 2 (the data
//                   gradient of a stride-2 convolution: a stride-1
//                   convolution of the zero-dilated output gradient).
// Out-of-range positions are the zero padding.
template <int MT, bool DILATE>
__global__ void __launch_bounds__(256) conv_mfma_kernel(const float* __restrict__ x, const uint16_t* __restrict__ wpk,
                                                       const float* __restrict__ bias, float* __restrict__ y, int C,
                                                       int C8, int Co, int KP, int Zi, int Yi, int Xi, int Zo, int Yo,
                                                       int Xo, int s, int act, int accumulate) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int b = blockIdx.y;
    const int nvo = Zo * Yo * Xo;
    const int v0 = (blockIdx.x * 4 + wave) * 16;
    if (v0 >= nvo) return;   // no block-level synchronisation follows
    const int col = lane & 15, kg = lane >> 4;
    const int v = v0 + col;
    const bool vok = v < nvo;
    const int vv = vok ? v : v0;
    const int xo = vv % Xo, yo = (vv / Xo) % Yo, zo = vv / (Xo * Yo);
    const size_t plane = (size_t)Zi * Yi * Xi;
    const float* xb = x + (size_t)b * C * plane;
    f32x4 acc[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) acc[mt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    const int nsteps = KP / 32;
    // this lane's K values of step st start at kk = 32 st + 8 kg = tap C8 + c0;
    // (tap, c0) and the tap's (kz, ky, kx) are advanced step by step
    int tap = (8 * kg) / C8, c0 = 8 * kg - tap * C8;
    int kz = tap / 9, ky = (tap / 3) % 3, kx = tap % 3;
    for (int st = 0; st < nsteps; ++st) {
        if (st > 0) {
            c0 += 32;
            while (c0 >= C8) {
                c0 -= C8;
                ++tap;
                if (++kx == 3) {
                    kx = 0;
                    if (++ky == 3) {
                        ky = 0;
                        ++kz;
                    }
                }
            }
        }
        const int kk0 = st * 32 + 8 * kg;
        int zi, yi, xi;
        bool ok = vok && tap < 27;
        if (!DILATE) {
            zi = s * zo + kz - 1;
            yi = s * yo + ky - 1;
            xi = s * xo + kx - 1;
        } else {
            const int pz = zo + kz - 1, py = yo + ky - 1, px = xo + kx - 1;
            ok = ok && pz >= 0 && py >= 0 && px >= 0 && !((pz | py | px) & 1);
            zi = pz >> 1;
            yi = py >> 1;
            xi = px >> 1;
        }
        ok = ok && zi >= 0 && zi < Zi && yi >= 0 && yi < Yi && xi >= 0 && xi < Xi;
        const float* xp = xb + (ok ? (size_t)c0 * plane + ((size_t)zi * Yi + yi) * Xi + xi : 0);
        bf16x8 bh, bl;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int c = c0 + j;
            const float val = (ok && c < C) ? xp[(size_t)j * plane] : 0.0f;
            __bf16 h, l;
            split_bf16(val, h, l);
            bh[j] = h;
            bl[j] = l;
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const bf16x8 a = *reinterpret_cast<const bf16x8*>(wpk + (size_t)(mt * 16 + col) * KP + kk0);
            acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bh, acc[mt], 0, 0, 0);
            acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bl, acc[mt], 0, 0, 0);
        }
    }
    if (!vok) return;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int o = mt * 16 + 4 * kg + r;
            if (o >= Co) continue;
            float val = acc[mt][r] + (bias ? bias[o] : 0.0f);
            if (act && val <= 0.0f) val *= kSlope;
            float* dst = y + ((size_t)b * Co + o) * nvo + v;
            *dst = accumulate ? *dst + val : val;
        }
}

// dst[b][v][c] = src[b][c][v] for c < C, 0 for C <= c < Cp (channels last,
// padded): tiles of 64 voxels through LDS so that both sides are coalesced.
__global__ void __launch_bounds__(256) to_channels_last_kernel(const float* __restrict__ src, float* __restrict__ dst,
                                                              int C, int Cp, int nv) {
    __shared__ float tile[64][65];
    const int b = blockIdx.y;
    const int v0 = blockIdx.x * 64;
    const int tid = threadIdx.x;
    for (int k = tid; k < Cp * 64; k += 256) {
        const int c = k / 64, vl = k - c * 64;
        tile[vl][c] = (c < C && v0 + vl < nv) ? src[((size_t)b * C + c) * nv + v0 + vl] : 0.0f;
    }
    __syncthreads();
    for (int k = tid; k < Cp * 64; k += 256) {
        const int vl = k / Cp, c = k - vl * Cp;
        if (v0 + vl < nv) dst[((size_t)b * nv + v0 + vl) * Cp + c] = tile[vl][c];
    }
}

// Weight and bias gradient as an implicit GEMM over the voxels of the batch:
// part[kc][o][n] = sum over chunk kc of the voxels t = (b, v) of
// gout[t][o] X[n][t] with n = tap * C16 + c (C16 = input channels rounded to
// 16), X[n][t] = x[b][s v + k - 1][c] (zero padding), and the bias column
// n = 27 C16 with X = 1.  Both operands are read channels last (x as
// [b][voxel][C16], gout as [t][MP]), so the 16 channels of a tile are 64
// contiguous bytes.  A wavefront owns 16 output channels (one tile), 16
// input channels, the nine taps of one kz and a chunk of voxels: per K step
// of 32 voxels it loads and splits its gout tile once and uses it for the
// nine taps (voxel coordinates and bounds are worked out once per step; each
// tap adds a constant offset).  Within a K step, element j of lane group kg
// is voxel 4 j + kg (the same order for both operands).  Both operands are
// split into BF16 pairs and the three leading products accumulated
// (g x = gh xh + gh xl + gl xh up to 2^-16 relative).  wgrad_reduce_kernel
// adds the chunks in fixed order.
__global__ void __launch_bounds__(256) wgrad_mfma_kernel(const float* __restrict__ xcl, const float* __restrict__ gcl,
                                                        float* __restrict__ part, int64_t K, int chunk, int nchunks,
                                                        int C16, int NP, int MP, int Zi, int Yi, int Xi, int Zo, int Yo,
                                                        int Xo, int s) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int kc = blockIdx.x * 4 + wave;
    if (kc >= nchunks) return;   // no block-level synchronisation follows
    const int cg = blockIdx.y / 3, kz = blockIdx.y - cg * 3;
    const int mt = blockIdx.z;
    const int col = lane & 15, kg = lane >> 4;
    const int o = mt * 16 + col;                 // row of the gout operand
    const int c = cg * 16 + col;                 // input channel of this lane's X column
    const bool bias = cg == 0 && kz == 0;        // this wavefront also forms the bias column
    const int nvo = Zo * Yo * Xo;
    const int64_t nvi = (int64_t)Zi * Yi * Xi;
    const int64_t t_begin = (int64_t)kc * chunk;
    const int64_t t_end = t_begin + chunk < K ? t_begin + chunk : K;
    f32x4 acc[9], accb = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int k = 0; k < 9; ++k) acc[k] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    bf16x8 ones;
#pragma unroll
    for (int j = 0; j < 8; ++j) ones[j] = (__bf16)(col == 0 ? 1.0f : 0.0f);
    for (int64_t t0 = t_begin; t0 < t_end; t0 += 32) {
        const int64_t t = t0 + kg;
        int b = (int)(t / nvo);
        int v = (int)(t - (int64_t)b * nvo);
        int xo = v % Xo, yo = (v / Xo) % Yo, zo = v / (Xo * Yo);
        bf16x8 gh, gl;
        int64_t base[8];        // index of (zi, yi, xi) = (s zo + kz - 1, s yo - 1, s xo - 1), channel c
        unsigned okm[8];        // bit ky: row s yo + ky - 1 in range; bit 3 + kx: column in range
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const bool tin = t + 4 * j < t_end;
            const float g = tin ? gcl[(t + 4 * j) * MP + o] : 0.0f;
            __bf16 h, l;
            split_bf16(g, h, l);
            gh[j] = h;
            gl[j] = l;
            const int zi = s * zo + kz - 1, yi0 = s * yo - 1, xi0 = s * xo - 1;
            unsigned m = 0;
            if (tin && zi >= 0 && zi < Zi) {
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    if (yi0 + k >= 0 && yi0 + k < Yi) m |= 1u << k;
                    if (xi0 + k >= 0 && xi0 + k < Xi) m |= 8u << k;
                }
            }
            okm[j] = m;
            base[j] = ((int64_t)b * nvi + ((int64_t)zi * Yi + yi0) * Xi + xi0) * C16 + c;
            // four voxels on (the order of the batch: b, then z, y, x)
            xo += 4;
            while (xo >= Xo) {
                xo -= Xo;
                if (++yo == Yo) {
                    yo = 0;
                    if (++zo == Zo) zo = 0;
                }
            }
            v += 4;
            while (v >= nvo) {
                v -= nvo;
                ++b;
            }
        }
        if (bias) {
            accb = __builtin_amdgcn_mfma_f32_16x16x32_bf16(gh, ones, accb, 0, 0, 0);
            accb = __builtin_amdgcn_mfma_f32_16x16x32_bf16(gl, ones, accb, 0, 0, 0);
        }
#pragma unroll
        for (int ky = 0; ky < 3; ++ky)
#pragma unroll
            for (int kx = 0; kx < 3; ++kx) {
                bf16x8 xh, xl;
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const bool in = ((okm[j] >> ky) & 1u) && ((okm[j] >> (3 + kx)) & 1u);
                    const float xv = in ? xcl[base[j] + ((int64_t)ky * Xi + kx) * C16] : 0.0f;
                    __bf16 h, l;
                    split_bf16(xv, h, l);
                    xh[j] = h;
                    xl[j] = l;
                }
                f32x4& a = acc[ky * 3 + kx];
                a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(gh, xh, a, 0, 0, 0);
                a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(gh, xl, a, 0, 0, 0);
                a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(gl, xh, a, 0, 0, 0);
            }
    }
    // C tile: rows 4 kg + r (output channels), column col (input channel)
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int tap = kz * 9 + k;
#pragma unroll
        for (int r = 0; r < 4; ++r)
            part[((size_t)kc * MP + mt * 16 + 4 * kg + r) * NP + tap * C16 + cg * 16 + col] = acc[k][r];
    }
    if (bias)
#pragma unroll
        for (int r = 0; r < 4; ++r) part[((size_t)kc * MP + mt * 16 + 4 * kg + r) * NP + 27 * C16 + col] = accb[r];
}

// Sums the chunks of the weight-gradient partials: a block takes 64
// consecutive columns n of one row o; its four wavefronts add every fourth
// chunk (ascending), then the four sums are added in wavefront order (a fixed
// order: deterministic).  Column n = tap * C16 + c goes to dw[o][c][tap],
// column 27 C16 to db[o].
__global__ void __launch_bounds__(256) wgrad_reduce_kernel(const float* __restrict__ part, float* __restrict__ dw,
                                                          float* __restrict__ db, int nchunks, int C, int C16, int Co,
                                                          int NP, int MP) {
    __shared__ float red[4][64];
    const int o = blockIdx.y;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int n = blockIdx.x * 64 + lane;
    float sum = 0.0f;
    if (n < NP)
        for (int kc = w; kc < nchunks; kc += 4) sum += part[((size_t)kc * MP + o) * NP + n];
    red[w][lane] = sum;
    __syncthreads();
    if (w != 0 || n > 27 * C16) return;
    const float tot = red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane];
    if (n == 27 * C16) {
        db[o] = tot;
        return;
    }
    const int tap = n / C16, c = n - tap * C16;
    if (c < C) dw[((size_t)o * C + c) * 27 + tap] = tot;
}

unsigned grid1(int64_t n, int bs = 256) { return (unsigned)std::max<int64_t>(1, (n + bs - 1) / bs); }

// splitmix64: a counter-based generator for the initial weights
uint64_t splitmix64(uint64_t& s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace

std::vector<NetLayer> net_layers(const int widths[3]) {
    const int c0 = widths[0], c1 = widths[1], c2 = widths[2];
    // {cin, cout, stride, act, level of the input}
    const int spec[12][5] = {{3, c0, 1, 1, 0},  {c0, c0, 1, 1, 0}, {c0, c1, 2, 1, 0}, {c1, c1, 1, 1, 1},
                             {c1, c2, 2, 1, 1}, {c2, c2, 1, 1, 2}, {c2, c2, 1, 1, 2}, {c2, c1, 1, 1, 2},
                             {c1, c1, 1, 1, 1}, {c1, c0, 1, 1, 1}, {c0, c0, 1, 1, 0}, {c0, 1, 1, 0, 0}};
    std::vector<NetLayer> L(12);
    int64_t off = 0;
    for (int k = 0; k < 12; ++k) {
        L[k].cin = spec[k][0];
        L[k].cout = spec[k][1];
        L[k].stride = spec[k][2];
        L[k].act = spec[k][3];
        L[k].level_in = spec[k][4];
        L[k].w_off = off;
        off += (int64_t)L[k].cout * L[k].cin * 27;
        L[k].b_off = off;
        off += L[k].cout;
    }
    return L;
}

namespace {

int round_up(int v, int m) { return (v + m - 1) / m * m; }

// Packed weight layouts of one layer (see pack_weights_kernel).
struct PackInfo {
    int c8in = 0, kpf = 0, rowsf = 0;   // forward: C8 = cin rounded to 8, K padded to 32, cout rounded to 16
    int c8out = 0, kpb = 0, rowsb = 0;  // data gradient: C8 = cout rounded to 8, rows = cin rounded to 16
    int64_t off_f = 0, off_b = 0;       // offsets into the packed buffer (multiples of 32 values)
};

std::vector<PackInfo> pack_layout(const std::vector<NetLayer>& layers, int64_t* total) {
    std::vector<PackInfo> pk(layers.size());
    int64_t off = 0;
    for (size_t k = 0; k < layers.size(); ++k) {
        const NetLayer& L = layers[k];
        PackInfo& q = pk[k];
        q.c8in = round_up(L.cin, 8);
        q.kpf = round_up(27 * q.c8in, 32);
        q.rowsf = round_up(L.cout, 16);
        q.c8out = round_up(L.cout, 8);
        q.kpb = round_up(27 * q.c8out, 32);
        q.rowsb = round_up(L.cin, 16);
        q.off_f = off;
        off += (int64_t)q.rowsf * q.kpf;
        q.off_b = off;
        off += (int64_t)q.rowsb * q.kpb;
    }
    *total = off;
    return pk;
}

// y (+)= conv of x with packed weights (rows = output channels, padded to
// 16 * mt): one wavefront per 16 output voxels
void conv_mfma(const float* x, const uint16_t* wpk, const float* bias, float* y, int B, int C, int C8, int Co,
               int KP, int rows, const int in[3], const int out[3], int s, bool dilate, int act, int accumulate,
               hipStream_t st) {
    const int nvo = out[0] * out[1] * out[2];
    dim3 grid((unsigned)((nvo + 63) / 64), (unsigned)B);
    const int mt = rows / 16;
#define SNSW_CONV_MFMA(MT, DIL)                                                                                    \
    hipLaunchKernelGGL((conv_mfma_kernel<MT, DIL>), grid, dim3(256), 0, st, x, wpk, bias, y, C, C8, Co, KP, in[0], \
                       in[1], in[2], out[0], out[1], out[2], s, act, accumulate)
    if (dilate) {
        if (mt == 1) SNSW_CONV_MFMA(1, true);
        else if (mt == 2) SNSW_CONV_MFMA(2, true);
        else if (mt == 3) SNSW_CONV_MFMA(3, true);
        else SNSW_CONV_MFMA(4, true);
    } else {
        if (mt == 1) SNSW_CONV_MFMA(1, false);
        else if (mt == 2) SNSW_CONV_MFMA(2, false);
        else if (mt == 3) SNSW_CONV_MFMA(3, false);
        else SNSW_CONV_MFMA(4, false);
    }
#undef SNSW_CONV_MFMA
    HIP_OK(hipGetLastError());
}

// Weight-gradient GEMM of a layer: input channels per tap rounded to 16,
// columns 27 C16 + 16 (the bias column and padding), wavefronts per chunk
// (16-channel groups x 3 kz x output-channel tiles), voxels per chunk (about
// 4096 wavefronts, at least 512 voxels each, a multiple of 32).
struct WgradShape {
    int C16, NP, MP, groups;
    int64_t chunk;
    int nchunks;
};
WgradShape wgrad_shape(const NetLayer& L, const PackInfo& q, int64_t K) {
    WgradShape w;
    w.C16 = round_up(L.cin, 16);
    w.NP = 27 * w.C16 + 16;
    w.MP = q.rowsf;
    w.groups = (w.C16 / 16) * 3 * (w.MP / 16);
    const int64_t want = std::max<int64_t>(1, 4096 / w.groups);
    w.chunk = std::max<int64_t>(512, ((K + want - 1) / want + 31) / 32 * 32);
    w.nchunks = (int)((K + w.chunk - 1) / w.chunk);
    return w;
}

}  // namespace

}  // namespace snsw

using namespace snsw;

// Tensor ids of the forward pass (activations kept for the backward pass).
enum : int { T_E0A, T_S0, T_E1A, T_S1, T_E2A, T_E2B, T_E2C, T_U1A, T_H1, T_U1B, T_U0A, T_H0, T_U0B, T_Y, T_COUNT };

struct snsw_net {
    snsw_ctx* ctx = nullptr;
    int widths[3] = {16, 32, 32};
    std::vector<NetLayer> layers;
    int64_t n_params = 0;
    float* theta = nullptr;      // FP32 masters
    float* m = nullptr;
    float* v = nullptr;
    float* grad = nullptr;
    uint16_t* wbf = nullptr;     // BF16 copy of the parameters (weights as the convolutions see them)
    uint16_t* wpk = nullptr;     // BF16 weights packed for the implicit-GEMM convolutions
    std::vector<PackInfo> pk;    // per layer: packed layouts (forward and data gradient)
    int64_t adam_t = 0;
    // workspace for the current shape
    int B = 0, dims[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    std::vector<float*> act;     // T_COUNT activations
    std::vector<float*> gact;    // their gradients
    float* gx_tmp = nullptr;     // gradient of the input when not requested
    float* wg_part = nullptr;    // weight-gradient partial sums per voxel chunk
    int64_t wg_cap = 0;          // its capacity (floats)
    float* cl_x = nullptr;       // channels-last copies of a layer's input and output gradient
    float* cl_g = nullptr;
    int64_t cl_cap = 0;          // capacity of each (floats)
    const float* x_in = nullptr; // input of the last forward pass
    double* loss_dev = nullptr;
    // source-iteration workspace
    int64_t si_E = 0;
    double* si_avg = nullptr;
    unsigned long long* si_max = nullptr;
    float* si_x = nullptr;
    float* si_y = nullptr;
};

namespace {

void free_ws(snsw_net* net) {
    for (float*& p : net->act)
        if (p) (void)hipFree(p), p = nullptr;
    for (float*& p : net->gact)
        if (p) (void)hipFree(p), p = nullptr;
    if (net->gx_tmp) (void)hipFree(net->gx_tmp);
    net->gx_tmp = nullptr;
    if (net->wg_part) (void)hipFree(net->wg_part);
    net->wg_part = nullptr;
    net->wg_cap = 0;
    if (net->cl_x) (void)hipFree(net->cl_x);
    if (net->cl_g) (void)hipFree(net->cl_g);
    net->cl_x = net->cl_g = nullptr;
    net->cl_cap = 0;
    net->B = 0;
}

int level_of_tensor(int t) {
    switch (t) {
        case T_E0A: case T_S0: case T_H0: case T_U0B: case T_Y: return 0;
        case T_E1A: case T_S1: case T_H1: case T_U1B: case T_U0A: return 1;
        default: return 2;
    }
}

int chans_of_tensor(const snsw_net* n, int t) {
    const int c0 = n->widths[0], c1 = n->widths[1], c2 = n->widths[2];
    switch (t) {
        case T_E0A: case T_S0: case T_H0: case T_U0B: case T_U0A: return c0;
        case T_E1A: case T_S1: case T_H1: case T_U1B: case T_U1A: return c1;
        case T_Y: return 1;
        default: return c2;
    }
}

int64_t tensor_len(const snsw_net* n, int t) {
    const int* d = n->dims[level_of_tensor(t)];
    return (int64_t)n->B * chans_of_tensor(n, t) * d[0] * d[1] * d[2];
}

void ensure_ws(snsw_net* net, int B, int Z, int Y, int X) {
    if (net->B == B && net->dims[0][0] == Z && net->dims[0][1] == Y && net->dims[0][2] == X) return;
    HIP_OK(hipStreamSynchronize(static_cast<hipStream_t>(net->ctx->stream)));
    free_ws(net);
    net->act.assign(T_COUNT, nullptr);
    net->gact.assign(T_COUNT, nullptr);
    net->B = B;
    int d[3] = {Z, Y, X};
    for (int l = 0; l < 3; ++l) {
        for (int a = 0; a < 3; ++a) net->dims[l][a] = d[a];
        for (int a = 0; a < 3; ++a) d[a] = out_size(d[a], 2);
    }
    for (int t = 0; t < T_COUNT; ++t) {
        HIP_OK(hipMalloc(&net->act[t], tensor_len(net, t) * sizeof(float)));
        HIP_OK(hipMalloc(&net->gact[t], tensor_len(net, t) * sizeof(float)));
    }
    HIP_OK(hipMalloc(&net->gx_tmp, (size_t)B * 3 * Z * Y * X * sizeof(float)));
    int64_t cap = 0, clcap = 0;
    for (size_t k = 0; k < net->layers.size(); ++k) {
        const NetLayer& L = net->layers[k];
        const int lout = L.stride == 2 ? L.level_in + 1 : L.level_in;
        const int64_t K = (int64_t)B * net->dims[lout][0] * net->dims[lout][1] * net->dims[lout][2];
        const WgradShape w = wgrad_shape(L, net->pk[k], K);
        cap = std::max(cap, (int64_t)w.nchunks * w.MP * w.NP);
        const int64_t Kin = (int64_t)B * net->dims[L.level_in][0] * net->dims[L.level_in][1] * net->dims[L.level_in][2];
        clcap = std::max(clcap, std::max(Kin * w.C16, K * w.MP));
    }
    HIP_OK(hipMalloc(&net->wg_part, cap * sizeof(float)));
    net->wg_cap = cap;
    HIP_OK(hipMalloc(&net->cl_x, clcap * sizeof(float)));
    HIP_OK(hipMalloc(&net->cl_g, clcap * sizeof(float)));
    net->cl_cap = clcap;
}

// conv layer k: input tensor (or x), output tensor
struct Wiring {
    int in, out;   // tensor ids (-1 = network input)
};
const Wiring kWire[12] = {{-1, T_E0A}, {T_E0A, T_S0}, {T_S0, T_E1A}, {T_E1A, T_S1}, {T_S1, T_E2A}, {T_E2A, T_E2B},
                          {T_E2B, T_E2C}, {T_E2C, T_U1A}, {T_H1, T_U1B}, {T_U1B, T_U0A}, {T_H0, T_U0B}, {T_U0B, T_Y}};

void run_conv(snsw_net* net, int k, const float* x, hipStream_t s) {
    const NetLayer& L = net->layers[k];
    const PackInfo& q = net->pk[k];
    const float* in = kWire[k].in < 0 ? x : net->act[kWire[k].in];
    const int lin = L.level_in, lout = L.stride == 2 ? lin + 1 : lin;
    conv_mfma(in, net->wpk + q.off_f, net->theta + L.b_off, net->act[kWire[k].out], net->B, L.cin, q.c8in, L.cout,
              q.kpf, q.rowsf, net->dims[lin], net->dims[lout], L.stride, false, L.act, 0, s);
}

// refreshes the packed weights from the FP32 masters (after any change)
void pack_weights(snsw_net* net, hipStream_t s) {
    for (size_t k = 0; k < net->layers.size(); ++k) {
        const NetLayer& L = net->layers[k];
        const PackInfo& q = net->pk[k];
        hipLaunchKernelGGL(pack_weights_kernel, dim3(grid1((int64_t)q.rowsf * q.kpf)), dim3(256), 0, s,
                           net->theta + L.w_off, net->wpk + q.off_f, L.cout, L.cin, q.rowsf, q.kpf, q.c8in, 0);
        HIP_OK(hipGetLastError());
        hipLaunchKernelGGL(pack_weights_kernel, dim3(grid1((int64_t)q.rowsb * q.kpb)), dim3(256), 0, s,
                           net->theta + L.w_off, net->wpk + q.off_b, L.cout, L.cin, q.rowsb, q.kpb, q.c8out, 1);
        HIP_OK(hipGetLastError());
    }
}

void run_upadd(snsw_net* net, int low, int skip, int out, hipStream_t s) {
    const int lh = level_of_tensor(out), ll = level_of_tensor(low);
    const int* D = net->dims[lh];
    const int* d = net->dims[ll];
    const int BC = net->B * chans_of_tensor(net, out);
    hipLaunchKernelGGL(upsample_add_kernel, dim3(grid1((int64_t)BC * D[0] * D[1] * D[2])), dim3(256), 0, s,
                       net->act[low], net->act[skip], net->act[out], BC, D[0], D[1], D[2], d[0], d[1], d[2]);
    HIP_OK(hipGetLastError());
}

void forward(snsw_net* net, const float* x, hipStream_t s) {
    net->x_in = x;
    for (int k = 0; k < 8; ++k) run_conv(net, k, x, s);
    run_upadd(net, T_U1A, T_S1, T_H1, s);
    run_conv(net, 8, x, s);
    run_conv(net, 9, x, s);
    run_upadd(net, T_U0A, T_S0, T_H0, s);
    run_conv(net, 10, x, s);
    run_conv(net, 11, x, s);
}

// Backward of conv layer k given the gradient of its output in gact[out]
// (masked here by the activation); writes (or adds to) the gradient of its
// input and the layer's parameter gradients.
void back_conv(snsw_net* net, int k, float* gin, int accumulate, hipStream_t s) {
    const NetLayer& L = net->layers[k];
    const int lin = L.level_in, lout = L.stride == 2 ? lin + 1 : lin;
    float* gout = net->gact[kWire[k].out];
    const float* yout = net->act[kWire[k].out];
    const int* di = net->dims[lin];
    const int* dout = net->dims[lout];
    const int64_t nout = (int64_t)net->B * L.cout * dout[0] * dout[1] * dout[2];
    if (L.act) {
        hipLaunchKernelGGL(act_backward_kernel, dim3(grid1(nout)), dim3(256), 0, s, yout, gout, nout);
        HIP_OK(hipGetLastError());
    }
    const float* in = kWire[k].in < 0 ? net->x_in : net->act[kWire[k].in];
    const PackInfo& q = net->pk[k];
    {
        const int64_t K = (int64_t)net->B * dout[0] * dout[1] * dout[2];
        const WgradShape w = wgrad_shape(L, q, K);
        if ((int64_t)w.nchunks * w.MP * w.NP > net->wg_cap)
            throw Error(SNSW_E_STATE, "weight-gradient workspace too small");
        const int nvi = di[0] * di[1] * di[2], nvo = dout[0] * dout[1] * dout[2];
        if ((int64_t)net->B * nvi * w.C16 > net->cl_cap || K * w.MP > net->cl_cap)
            throw Error(SNSW_E_STATE, "channels-last workspace too small");
        hipLaunchKernelGGL(to_channels_last_kernel, dim3((unsigned)((nvi + 63) / 64), (unsigned)net->B), dim3(256), 0,
                           s, in, net->cl_x, L.cin, w.C16, nvi);
        HIP_OK(hipGetLastError());
        hipLaunchKernelGGL(to_channels_last_kernel, dim3((unsigned)((nvo + 63) / 64), (unsigned)net->B), dim3(256), 0,
                           s, gout, net->cl_g, L.cout, w.MP, nvo);
        HIP_OK(hipGetLastError());
        dim3 grid((unsigned)((w.nchunks + 3) / 4), (unsigned)(w.C16 / 16 * 3), (unsigned)(w.MP / 16));
        hipLaunchKernelGGL(wgrad_mfma_kernel, grid, dim3(256), 0, s, net->cl_x, net->cl_g, net->wg_part, K,
                           (int)w.chunk, w.nchunks, w.C16, w.NP, w.MP, di[0], di[1], di[2], dout[0], dout[1], dout[2],
                           L.stride);
        HIP_OK(hipGetLastError());
        hipLaunchKernelGGL(wgrad_reduce_kernel, dim3((unsigned)((w.NP + 63) / 64), (unsigned)L.cout), dim3(256), 0,
                           s, net->wg_part, net->grad + L.w_off, net->grad + L.b_off, w.nchunks, L.cin, w.C16, L.cout,
                           w.NP, w.MP);
        HIP_OK(hipGetLastError());
    }
    // data gradient: a convolution of gout with the mirrored, transposed
    // weights (stride 2: over the zero-dilated gout)
    if (gin)
        conv_mfma(gout, net->wpk + q.off_b, nullptr, gin, net->B, L.cout, q.c8out, L.cin, q.kpb, q.rowsb, dout, di, 1,
                  L.stride == 2, 0, accumulate, s);
}

void upadd_back(snsw_net* net, int h, int low, hipStream_t s) {
    const int* D = net->dims[level_of_tensor(h)];
    const int* d = net->dims[level_of_tensor(low)];
    const int BC = net->B * chans_of_tensor(net, h);
    hipLaunchKernelGGL(upsample_back_kernel, dim3(grid1((int64_t)BC * d[0] * d[1] * d[2])), dim3(256), 0, s,
                       net->gact[h], net->gact[low], BC, D[0], D[1], D[2], d[0], d[1], d[2]);
    HIP_OK(hipGetLastError());
}

void backward(snsw_net* net, const float* dy, float* dx, hipStream_t s) {
    HIP_OK(hipMemcpyAsync(net->gact[T_Y], dy, tensor_len(net, T_Y) * sizeof(float), hipMemcpyDeviceToDevice, s));
    back_conv(net, 11, net->gact[T_U0B], 0, s);
    back_conv(net, 10, net->gact[T_H0], 0, s);          // gradient of h0 = gradient of skip s0
    upadd_back(net, T_H0, T_U0A, s);
    back_conv(net, 9, net->gact[T_U1B], 0, s);
    back_conv(net, 8, net->gact[T_H1], 0, s);           // gradient of h1 = gradient of skip s1
    upadd_back(net, T_H1, T_U1A, s);
    back_conv(net, 7, net->gact[T_E2C], 0, s);
    back_conv(net, 6, net->gact[T_E2B], 0, s);
    back_conv(net, 5, net->gact[T_E2A], 0, s);
    back_conv(net, 4, net->gact[T_H1], 1, s);           // s1 gets both paths
    HIP_OK(hipMemcpyAsync(net->gact[T_S1], net->gact[T_H1], tensor_len(net, T_S1) * sizeof(float),
                          hipMemcpyDeviceToDevice, s));
    back_conv(net, 3, net->gact[T_E1A], 0, s);
    back_conv(net, 2, net->gact[T_H0], 1, s);           // s0 gets both paths
    HIP_OK(hipMemcpyAsync(net->gact[T_S0], net->gact[T_H0], tensor_len(net, T_S0) * sizeof(float),
                          hipMemcpyDeviceToDevice, s));
    back_conv(net, 1, net->gact[T_E0A], 0, s);
    back_conv(net, 0, dx ? dx : net->gx_tmp, 0, s);
}

void net_release(snsw_net* net) noexcept {
    if (!net) return;
    (void)hipStreamSynchronize(static_cast<hipStream_t>(net->ctx->stream));
    free_ws(net);
    void* ptrs[] = {net->theta, net->m, net->v, net->grad, net->wbf, net->wpk, net->loss_dev,
                    net->si_avg, net->si_max, net->si_x, net->si_y};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    delete net;
}

void ensure_si_ws(snsw_net* net, int64_t E) {
    if (net->si_E == E) return;
    HIP_OK(hipStreamSynchronize(static_cast<hipStream_t>(net->ctx->stream)));
    void* ptrs[] = {net->si_avg, net->si_max, net->si_x, net->si_y};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    net->si_avg = nullptr;
    net->si_max = nullptr;
    net->si_x = nullptr;
    net->si_y = nullptr;
    net->si_E = 0;
    HIP_OK(hipMalloc(&net->si_avg, E * sizeof(double)));
    HIP_OK(hipMalloc(&net->si_max, 2 * sizeof(unsigned long long)));
    HIP_OK(hipMalloc(&net->si_x, 3 * E * sizeof(float)));
    HIP_OK(hipMalloc(&net->si_y, E * sizeof(float)));
    net->si_E = E;
}

void grid_of(const HostProblem& hp, int g[3]) {
    // (Z, Y, X) element grid, element e = i + nx (j + ny k)
    g[0] = hp.dim == 3 ? hp.nx[2] : 1;
    g[1] = hp.nx[1];
    g[2] = hp.nx[0];
}

}  // namespace

namespace snsw {

void net_apply_correction(snsw_net* net, snsw_problem* prob, const double* phi_prev, double* phi_swept) {
    DeviceProblem* dp = need_device(prob);
    const HostProblem& hp = prob->hp;
    hipStream_t s = dp->stream;
    ensure_si_ws(net, hp.E);
    int g[3];
    grid_of(hp, g);
    ensure_ws(net, 1, g[0], g[1], g[2]);
    HIP_OK(hipMemsetAsync(net->si_max, 0, sizeof(unsigned long long), s));
    hipLaunchKernelGGL(elem_avg_kernel, dim3(grid1(hp.E)), dim3(256), 0, s, dp->geo, hp.dim, hp.n, hp.E,
                       phi_swept, phi_prev, net->si_avg, net->si_max);
    HIP_OK(hipGetLastError());
    hipLaunchKernelGGL(net_input_kernel, dim3(grid1(hp.E)), dim3(256), 0, s, net->si_avg, net->si_max, dp->sigma_t,
                       dp->sigma_s, hp.E, net->si_x);
    HIP_OK(hipGetLastError());
    forward(net, net->si_x, s);
    hipLaunchKernelGGL(apply_correction_kernel, dim3(grid1(hp.E * hp.n)), dim3(256), 0, s, phi_swept,
                       net->act[T_Y], net->si_max, hp.n, hp.E);
    HIP_OK(hipGetLastError());
}

// Scratch of snsw_learn_pair_noalloc: the two element-mean vectors and the
// max-bits counter live in a file-scope device array (one copy per GPU, held
// until the process ends) instead of per-call allocations.  Layout in
// doubles: [0] max counter (u64 bits), [1..31] unused (keeps the vectors on
// a 256-byte boundary), [32, 32 + E) residual means, [32 + E, 32 + 2E)
// target means.
constexpr int64_t kNoAllocMaxE = int64_t(1) << 20;
constexpr int64_t kNoAllocHead = 32;
static __device__ __align__(256) double scratch[kNoAllocHead + 2 * kNoAllocMaxE];

namespace {

__global__ void clear_u64_kernel(unsigned long long* p) { *p = 0ull; }

// Device address of `scratch` on each device, taken once per device with
// that device current (the array's host-side name is not a device address).
std::mutex g_scratch_mu;
double* g_scratch_ptr[64] = {};

double* scratch_on(int device) {
    if (device < 0 || device >= 64) throw Error(SNSW_E_INVALID_ARG, "device id out of range for the static scratch");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        HIP_OK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) throw Error(SNSW_E_HIP, "hipGetSymbolAddress returned no address for the scratch array");
        g_scratch_ptr[device] = static_cast<double*>(ptr);
    }
    return g_scratch_ptr[device];
}

}  // namespace

}  // namespace snsw

extern "C" {

int snsw_net_create(snsw_ctx* ctx, const snsw_net_desc* desc, snsw_net** out) {
    snsw_net* net = nullptr;
    const int rc = snsw_guard([&] {
        if (!ctx || !desc || !out) throw Error(SNSW_E_INVALID_ARG, "NULL argument");
        *out = nullptr;
        if (ctx->device < 0) throw Error(SNSW_E_UNSUPPORTED, "host-only context: no device work");
        for (int k = 0; k < 3; ++k)
            if (desc->widths[k] < 1 || desc->widths[k] > 64)
                throw Error(SNSW_E_INVALID_ARG, "network widths must lie in [1, 64]");
        DeviceGuard g(ctx->device);
        net = new snsw_net();
        net->ctx = ctx;
        for (int k = 0; k < 3; ++k) net->widths[k] = desc->widths[k];
        net->layers = net_layers(net->widths);
        net->n_params = net->layers.back().b_off + net->layers.back().cout;
        const int64_t P = net->n_params;
        HIP_OK(hipMalloc(&net->theta, P * sizeof(float)));
        HIP_OK(hipMalloc(&net->m, P * sizeof(float)));
        HIP_OK(hipMalloc(&net->v, P * sizeof(float)));
        HIP_OK(hipMalloc(&net->grad, P * sizeof(float)));
        HIP_OK(hipMalloc(&net->wbf, P * sizeof(uint16_t)));
        int64_t packed = 0;
        net->pk = pack_layout(net->layers, &packed);
        HIP_OK(hipMalloc(&net->wpk, packed * sizeof(uint16_t)));
        HIP_OK(hipMalloc(&net->loss_dev, (1 + kMseBlocks) * sizeof(double)));
        // He-uniform weights (output layer scaled by 0.1), zero biases
        std::vector<float> h(P, 0.0f);
        uint64_t st = desc->seed;
        for (const NetLayer& L : net->layers) {
            const double bound = std::sqrt(6.0 / (L.cin * 27.0)) * (L.act ? 1.0 : 0.1);
            for (int64_t t = 0; t < (int64_t)L.cout * L.cin * 27; ++t) {
                const double u = (double)(splitmix64(st) >> 11) * (1.0 / 9007199254740992.0);
                h[L.w_off + t] = (float)((2.0 * u - 1.0) * bound);
            }
        }
        hipStream_t s = static_cast<hipStream_t>(ctx->stream);
        HIP_OK(hipMemcpyAsync(net->theta, h.data(), P * sizeof(float), hipMemcpyHostToDevice, s));
        HIP_OK(hipMemsetAsync(net->m, 0, P * sizeof(float), s));
        HIP_OK(hipMemsetAsync(net->v, 0, P * sizeof(float), s));
        HIP_OK(hipMemsetAsync(net->grad, 0, P * sizeof(float), s));
        hipLaunchKernelGGL(to_bf16_kernel, dim3(grid1(P)), dim3(256), 0, s, net->theta, net->wbf, P);
        HIP_OK(hipGetLastError());
        pack_weights(net, s);
        HIP_OK(hipStreamSynchronize(s));
        *out = net;
    });
    if (rc != SNSW_OK && net) net_release(net);
    return rc;
}

void snsw_net_destroy(snsw_net* net) {
    if (!net) return;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(net->ctx->device);
    net_release(net);
    if (prev >= 0) (void)hipSetDevice(prev);
}

int snsw_net_n_params(const snsw_net* net, int64_t* n) {
    return snsw_guard([&] {
        if (!net || !n) throw Error(SNSW_E_INVALID_ARG, "NULL argument");
        *n = net->n_params;
    });
}

int snsw_net_get_params(const snsw_net* net, float* host) {
    return snsw_guard([&] {
        if (!net || !host) throw Error(SNSW_E_INVALID_ARG, "NULL argument");
        DeviceGuard g(net->ctx->device);
        hipStream_t s = static_cast<hipStream_t>(net->ctx->stream);
        HIP_OK(hipMemcpyAsync(host, net->theta, net->n_params * sizeof(float), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
    });
}

int snsw_net_set_params(snsw_net* net, const float* host) {
    return snsw_guard([&] {
        if (!net || !host) throw Error(SNSW_E_INVALID_ARG, "NULL argument");
        for (int64_t t = 0; t < net->n_params; ++t)
            if (!std::isfinite(host[t])) throw Error(SNSW_E_NONFINITE, "non-finite parameter");
        DeviceGuard g(net->ctx->device);
        hipStream_t s = static_cast<hipStream_t>(net->ctx->stream);
        const int64_t P = net->n_params;
        HIP_OK(hipMemcpyAsync(net->theta, host, P * sizeof(float), hipMemcpyHostToDevice, s));
        HIP_OK(hipMemsetAsync(net->m, 0, P * sizeof(float), s));
        HIP_OK(hipMemsetAsync(net->v, 0, P * sizeof(float), s));
        hipLaunchKernelGGL(to_bf16_kernel, dim3(grid1(P)), dim3(256), 0, s, net->theta, net->wbf, P);
        HIP_OK(hipGetLastError());
        pack_weights(net, s);
        HIP_OK(hipStreamSynchronize(s));
        net->adam_t = 0;
    });
}

int snsw_net_get_grads(const snsw_net* net, float* host) {
    return snsw_guard([&] {
        if (!net || !host) throw Error(SNSW_E_INVALID_ARG, "NULL argument");
        DeviceGuard g(net->ctx->device);
        hipStream_t s = static_cast<hipStream_t>(net->ctx->stream);
        HIP_OK(hipMemcpyAsync(host, net->grad, net->n_params * sizeof(float), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
    });
}

int snsw_net_forward(snsw_net* net, const float* d_x, float* d_y, int32_t batch, int32_t nz, int32_t ny, int32_t nx) {
    return snsw_guard([&] {
        if (!net || !d_x || !d_y) throw Error(SNSW_E_INVALID_ARG, "NULL argument");
        if (batch < 1 || nz < 1 || ny < 1 || nx < 1) throw Error(SNSW_E_SHAPE, "batch and grid sizes must be >= 1");
        DeviceGuard g(net->ctx->device);
        hipStream_t s = static_cast<hipStream_t>(net->ctx->stream);
        ensure_ws(net, batch, nz, ny, nx);
        forward(net, d_x, s);
        HIP_OK(hipMemcpyAsync(d_y, net->act[T_Y], tensor_len(net, T_Y) * sizeof(float), hipMemcpyDeviceToDevice, s));
    });
}

int snsw_net_loss(snsw_net* net, const float* d_y, const float* d_t, int64_t count, float* d_dy, double* loss) {
    return snsw_guard([&] {
        if (!net || !d_y || !d_t || !d_dy || !loss) throw Error(SNSW_E_INVALID_ARG, "NULL argument");
        if (count < 1) throw Error(SNSW_E_SHAPE, "count must be >= 1");
        DeviceGuard g(net->ctx->device);
        hipStream_t s = static_cast<hipStream_t>(net->ctx->stream);
        const int blocks = (int)std::min<int64_t>(kMseBlocks, (count + 255) / 256);
        hipLaunchKernelGGL(mse_partial_kernel, dim3(blocks), dim3(256), 0, s, d_y, d_t, count, d_dy, net->loss_dev + 1);
        HIP_OK(hipGetLastError());
        hipLaunchKernelGGL(mse_final_kernel, dim3(1), dim3(64), 0, s, net->loss_dev + 1, blocks, count, net->loss_dev);
        HIP_OK(hipGetLastError());
        HIP_OK(hipMemcpyAsync(loss, net->loss_dev, sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
    });
}

int snsw_net_backward(snsw_net* net, const float* d_dy, float* d_dx) {
    return snsw_guard([&] {
        if (!net || !d_dy) throw Error(SNSW_E_INVALID_ARG, "NULL argument");
        if (!net->x_in || net->B == 0) throw Error(SNSW_E_STATE, "backward needs a preceding forward pass");
        DeviceGuard g(net->ctx->device);
        backward(net, d_dy, d_dx, static_cast<hipStream_t>(net->ctx->stream));
    });
}

int snsw_net_step(snsw_net* net, const snsw_adam* opt) {
    return snsw_guard([&] {
        if (!net || !opt) throw Error(SNSW_E_INVALID_ARG, "NULL argument");
        if (!(opt->lr > 0.0f) || !(opt->beta1 >= 0.0f && opt->beta1 < 1.0f) ||
            !(opt->beta2 >= 0.0f && opt->beta2 < 1.0f) || !(opt->eps > 0.0f))
            throw Error(SNSW_E_INVALID_ARG, "bad Adam parameters");
        DeviceGuard g(net->ctx->device);
        hipStream_t s = static_cast<hipStream_t>(net->ctx->stream);
        ++net->adam_t;
        const float c1 = 1.0f - std::pow(opt->beta1, (float)net->adam_t);
        const float c2 = 1.0f - std::pow(opt->beta2, (float)net->adam_t);
        hipLaunchKernelGGL(adam_kernel, dim3(grid1(net->n_params)), dim3(256), 0, s, net->theta, net->grad, net->m,
                           net->v, net->wbf, net->n_params, opt->lr, opt->beta1, opt->beta2, opt->eps, c1, c2);
        HIP_OK(hipGetLastError());
        pack_weights(net, s);
    });
}

int snsw_learn_pair(snsw_problem* prob, const double* d_phi_prev, const double* d_phi_swept, const double* d_phi_star,
                    float* d_x, float* d_t) {
    return snsw_guard([&] {
        if (!d_phi_prev || !d_phi_swept || !d_x) throw Error(SNSW_E_INVALID_ARG, "NULL argument");
        DeviceProblem* dp = need_device(prob);
        const HostProblem& hp = prob->hp;
        DeviceGuard g(dp->device);
        hipStream_t s = dp->stream;
        double* avg = nullptr;
        unsigned long long* mx = nullptr;
        HIP_OK(hipMalloc(&avg, 2 * hp.E * sizeof(double)));
        HIP_OK(hipMalloc(&mx, 2 * sizeof(unsigned long long)));
        try {
            HIP_OK(hipMemsetAsync(mx, 0, 2 * sizeof(unsigned long long), s));
            hipLaunchKernelGGL(elem_avg_kernel, dim3(grid1(hp.E)), dim3(256), 0, s, dp->geo, hp.dim, hp.n, hp.E,
                               d_phi_swept, d_phi_prev, avg, mx);
            HIP_OK(hipGetLastError());
            hipLaunchKernelGGL(net_input_kernel, dim3(grid1(hp.E)), dim3(256), 0, s, avg, mx, dp->sigma_t,
                               dp->sigma_s, hp.E, d_x);
            HIP_OK(hipGetLastError());
            if (d_t && d_phi_star) {
                hipLaunchKernelGGL(elem_avg_kernel, dim3(grid1(hp.E)), dim3(256), 0, s, dp->geo, hp.dim, hp.n, hp.E,
                                   d_phi_star, d_phi_swept, avg + hp.E, nullptr);
                HIP_OK(hipGetLastError());
                hipLaunchKernelGGL(net_target_kernel, dim3(grid1(hp.E)), dim3(256), 0, s, avg + hp.E, mx, hp.E, d_t);
                HIP_OK(hipGetLastError());
            }
            HIP_OK(hipStreamSynchronize(s));
        } catch (...) {
            (void)hipFree(avg);
            (void)hipFree(mx);
            throw;
        }
        HIP_OK(hipFree(avg));
        HIP_OK(hipFree(mx));
    });
}

int snsw_learn_pair_noalloc(snsw_problem* prob, const double* d_phi_prev, const double* d_phi_swept,
                            const double* d_phi_star, float* d_x, float* d_t) {
    return snsw_guard([&] {
        if (!d_phi_prev || !d_phi_swept || !d_x) throw Error(SNSW_E_INVALID_ARG, "NULL argument");
        DeviceProblem* dp = need_device(prob);
        const HostProblem& hp = prob->hp;
        if (hp.E > kNoAllocMaxE)
            throw Error(SNSW_E_SHAPE, "snsw_learn_pair_noalloc: " + std::to_string(hp.E) +
                                          " elements exceed the static scratch's maximum of " +
                                          std::to_string(kNoAllocMaxE));
        DeviceGuard g(dp->device);
        hipStream_t s = dp->stream;
        double* base = scratch_on(dp->device);
        unsigned long long* mx = reinterpret_cast<unsigned long long*>(base);
        double* avg = base + kNoAllocHead;
        // the counter keeps the previous call's value: clear it with a kernel
        // (no memset node, so a captured call replays correctly)
        hipLaunchKernelGGL(clear_u64_kernel, dim3(1), dim3(1), 0, s, mx);
        HIP_OK(hipGetLastError());
        hipLaunchKernelGGL(elem_avg_kernel, dim3(grid1(hp.E)), dim3(256), 0, s, dp->geo, hp.dim, hp.n, hp.E,
                           d_phi_swept, d_phi_prev, avg, mx);
        HIP_OK(hipGetLastError());
        hipLaunchKernelGGL(net_input_kernel, dim3(grid1(hp.E)), dim3(256), 0, s, avg, mx, dp->sigma_t, dp->sigma_s,
                           hp.E, d_x);
        HIP_OK(hipGetLastError());
        if (d_t && d_phi_star) {
            hipLaunchKernelGGL(elem_avg_kernel, dim3(grid1(hp.E)), dim3(256), 0, s, dp->geo, hp.dim, hp.n, hp.E,
                               d_phi_star, d_phi_swept, avg + hp.E, nullptr);
            HIP_OK(hipGetLastError());
            hipLaunchKernelGGL(net_target_kernel, dim3(grid1(hp.E)), dim3(256), 0, s, avg + hp.E, mx, hp.E, d_t);
            HIP_OK(hipGetLastError());
        }
    });
}

}  // extern "C"
