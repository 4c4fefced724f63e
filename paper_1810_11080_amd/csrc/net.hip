// Learned source-iteration correction: a small 3D U-Net over the element
// grid (BF16 convolution weights, FP32 activations and accumulation, FP32
// master weights with Adam), its training kernels, and the kernels that turn
// a sweep's scalar-flux residual into network input and apply the network's
// correction (FP64).
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

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// float -> bfloat16, round to nearest even; NaN stays a quiet NaN
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (uint16_t)((u >> 16) | 0x0040u);
    const uint32_t bias = 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)((u + bias) >> 16);
}

__host__ __device__ inline int out_size(int n, int s) { return (n - 1) / s + 1; }

// y[b][o][v] = act(bias[o] + sum_{i,k} w[o][i][k] x[b][i][s v + k - 1]);
// block: blockDim.x output voxels x CO_T output channels, weights of the channel
// tile staged in LDS as FP32.
template <int CO_T>
__global__ void __launch_bounds__(256) conv_fwd_kernel(const float* __restrict__ x, const uint16_t* __restrict__ w,
                                                      const float* __restrict__ bias, float* __restrict__ y, int Ci,
                                                      int Co, int Z, int Y, int X, int Zo, int Yo, int Xo, int s,
                                                      int act) {
    extern __shared__ float wl[];   // [CO_T][Ci*27]
    const int o0 = blockIdx.y * CO_T;
    const int b = blockIdx.z;
    const int K = Ci * 27;
    for (int t = threadIdx.x; t < CO_T * K; t += blockDim.x) {
        const int oo = t / K, r = t - oo * K;
        wl[t] = (o0 + oo < Co) ? bf16_to_f32(w[(size_t)(o0 + oo) * K + r]) : 0.0f;
    }
    __syncthreads();
    const int nvo = Zo * Yo * Xo;
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nvo) return;
    const int xo = v % Xo, yo = (v / Xo) % Yo, zo = v / (Xo * Yo);
    float acc[CO_T];
#pragma unroll
    for (int t = 0; t < CO_T; ++t) acc[t] = (o0 + t < Co) ? bias[o0 + t] : 0.0f;
    const size_t plane = (size_t)Z * Y * X;
    for (int i = 0; i < Ci; ++i) {
        const float* xi = x + ((size_t)b * Ci + i) * plane;
        for (int kz = 0; kz < 3; ++kz) {
            const int z = s * zo + kz - 1;
            if (z < 0 || z >= Z) continue;
            for (int ky = 0; ky < 3; ++ky) {
                const int yy = s * yo + ky - 1;
                if (yy < 0 || yy >= Y) continue;
#pragma unroll
                for (int kx = 0; kx < 3; ++kx) {
                    const int xx = s * xo + kx - 1;
                    if (xx < 0 || xx >= X) continue;
                    const float xv = xi[((size_t)z * Y + yy) * X + xx];
                    const int k = i * 27 + kz * 9 + ky * 3 + kx;
#pragma unroll
                    for (int t = 0; t < CO_T; ++t) acc[t] += wl[t * K + k] * xv;
                }
            }
        }
    }
#pragma unroll
    for (int t = 0; t < CO_T; ++t) {
        if (o0 + t >= Co) break;
        float r = acc[t];
        if (act && r <= 0.0f) r *= kSlope;
        y[((size_t)b * Co + o0 + t) * nvo + v] = r;
    }
}

// g_in[b][i][u] (+)= sum_{o,k} w[o][i][k] g_out[b][o][(u + 1 - k)/s]
// over the k for which (u + 1 - k) is a non-negative multiple of s in range.
template <int CI_T>
__global__ void __launch_bounds__(256) conv_bwd_data_kernel(const float* __restrict__ gout,
                                                           const uint16_t* __restrict__ w, float* __restrict__ gin,
                                                           int Ci, int Co, int Z, int Y, int X, int Zo, int Yo,
                                                           int Xo, int s, int accumulate) {
    extern __shared__ float wl[];   // [CI_T][Co*27]
    const int i0 = blockIdx.y * CI_T;
    const int b = blockIdx.z;
    const int K = Co * 27;
    for (int t = threadIdx.x; t < CI_T * K; t += blockDim.x) {
        const int ii = t / K, r = t - ii * K;
        const int o = r / 27, k = r - o * 27;
        wl[t] = (i0 + ii < Ci) ? bf16_to_f32(w[((size_t)o * Ci + i0 + ii) * 27 + k]) : 0.0f;
    }
    __syncthreads();
    const int nv = Z * Y * X;
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= nv) return;
    const int xx = u % X, yy = (u / X) % Y, zz = u / (X * Y);
    float acc[CI_T];
#pragma unroll
    for (int t = 0; t < CI_T; ++t) acc[t] = 0.0f;
    const size_t plane = (size_t)Zo * Yo * Xo;
    for (int o = 0; o < Co; ++o) {
        const float* go = gout + ((size_t)b * Co + o) * plane;
        for (int kz = 0; kz < 3; ++kz) {
            const int nz = zz + 1 - kz;
            if (nz < 0 || nz % s) continue;
            const int zo = nz / s;
            if (zo >= Zo) continue;
            for (int ky = 0; ky < 3; ++ky) {
                const int ny = yy + 1 - ky;
                if (ny < 0 || ny % s) continue;
                const int yo = ny / s;
                if (yo >= Yo) continue;
                for (int kx = 0; kx < 3; ++kx) {
                    const int nx = xx + 1 - kx;
                    if (nx < 0 || nx % s) continue;
                    const int xo = nx / s;
                    if (xo >= Xo) continue;
                    const float g = go[((size_t)zo * Yo + yo) * Xo + xo];
                    const int k = o * 27 + kz * 9 + ky * 3 + kx;
#pragma unroll
                    for (int t = 0; t < CI_T; ++t) acc[t] += wl[t * K + k] * g;
                }
            }
        }
    }
#pragma unroll
    for (int t = 0; t < CI_T; ++t) {
        if (i0 + t >= Ci) break;
        float* dst = gin + ((size_t)b * Ci + i0 + t) * nv + u;
        *dst = accumulate ? *dst + acc[t] : acc[t];
    }
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// dw[o][i][k] = sum_{b,v} g_out[b][o][v] x[b][i][s v + k - 1]; one block per
// (o, i); the 27 partial sums of each thread are reduced across the block.
__global__ void __launch_bounds__(256) conv_bwd_weight_kernel(const float* __restrict__ x,
                                                             const float* __restrict__ gout, float* __restrict__ dw,
                                                             int B, int Ci, int Co, int Z, int Y, int X, int Zo,
                                                             int Yo, int Xo, int s) {
    __shared__ float red[4][27];
    const int o = blockIdx.x / Ci, i = blockIdx.x - (blockIdx.x / Ci) * Ci;
    const int nvo = Zo * Yo * Xo;
    const size_t plane = (size_t)Z * Y * X;
    float acc[27];
#pragma unroll
    for (int k = 0; k < 27; ++k) acc[k] = 0.0f;
    for (int64_t t = threadIdx.x; t < (int64_t)B * nvo; t += blockDim.x) {
        const int b = (int)(t / nvo), v = (int)(t - (int64_t)b * nvo);
        const float g = gout[((size_t)b * Co + o) * nvo + v];
        const int xo = v % Xo, yo = (v / Xo) % Yo, zo = v / (Xo * Yo);
        const float* xi = x + ((size_t)b * Ci + i) * plane;
#pragma unroll
        for (int kz = 0; kz < 3; ++kz) {
            const int z = s * zo + kz - 1;
#pragma unroll
            for (int ky = 0; ky < 3; ++ky) {
                const int yy = s * yo + ky - 1;
#pragma unroll
                for (int kx = 0; kx < 3; ++kx) {
                    const int xx = s * xo + kx - 1;
                    const bool in = z >= 0 && z < Z && yy >= 0 && yy < Y && xx >= 0 && xx < X;
                    const float xv = in ? xi[((size_t)z * Y + yy) * X + xx] : 0.0f;
                    acc[kz * 9 + ky * 3 + kx] += g * xv;
                }
            }
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 27; ++k) {
        const float r = wave_sum(acc[k]);
        if (lane == 0) red[wave][k] = r;
    }
    __syncthreads();
    if (threadIdx.x < 27) {
        const float r = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
        dw[((size_t)o * Ci + i) * 27 + threadIdx.x] = r;
    }
}

// db[o] = sum_{b,v} g_out[b][o][v]; one block per o
__global__ void __launch_bounds__(256) bias_grad_kernel(const float* __restrict__ gout, float* __restrict__ db, int B,
                                                       int Co, int nvo) {
    __shared__ float red[4];
    const int o = blockIdx.x;
    float acc = 0.0f;
    for (int64_t t = threadIdx.x; t < (int64_t)B * nvo; t += blockDim.x) {
        const int b = (int)(t / nvo), v = (int)(t - (int64_t)b * nvo);
        acc += gout[((size_t)b * Co + o) * nvo + v];
    }
    const float r = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = r;
    __syncthreads();
    if (threadIdx.x == 0) db[o] = red[0] + red[1] + red[2] + red[3];
}

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

// loss = mean((y - t)^2) (FP64 accumulation, one block), dy = 2 (y - t) / n
__global__ void __launch_bounds__(1024) mse_kernel(const float* __restrict__ y, const float* __restrict__ tgt,
                                                  int64_t n, float* __restrict__ dy, double* __restrict__ loss) {
    __shared__ double red[16];
    double acc = 0.0;
    const float scale = 2.0f / (float)n;
    for (int64_t t = threadIdx.x; t < n; t += blockDim.x) {
        const float d = y[t] - tgt[t];
        acc += (double)d * (double)d;
        dy[t] = scale * d;
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += red[k];
        *loss = s / (double)n;
    }
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

// Channel tile and block size: small grids take narrow channel tiles and
// small blocks so that the launch still spreads over many CUs.
struct ConvShape {
    int tile, threads;
};
ConvShape conv_shape(int64_t voxels, int K) {
    ConvShape c;
    c.tile = voxels >= 32768 ? 16 : (voxels >= 8192 ? 8 : 4);
    while (c.tile > 4 && (int64_t)c.tile * K * 4 > 64 * 1024) c.tile /= 2;
    c.threads = voxels >= 32768 ? 256 : 64;
    return c;
}

void conv_fwd(const float* x, const uint16_t* w, const float* bias, float* y, int B, int Ci, int Co, const int in[3],
              const int out[3], int s, int act, hipStream_t st) {
    const int nvo = out[0] * out[1] * out[2];
    const ConvShape c = conv_shape((int64_t)B * nvo, Ci * 27);
    const size_t lds = (size_t)c.tile * Ci * 27 * sizeof(float);
    dim3 grid(grid1(nvo, c.threads), (unsigned)((Co + c.tile - 1) / c.tile), (unsigned)B);
    if (c.tile == 16)
        hipLaunchKernelGGL(conv_fwd_kernel<16>, grid, dim3(c.threads), lds, st, x, w, bias, y, Ci, Co, in[0], in[1],
                           in[2], out[0], out[1], out[2], s, act);
    else if (c.tile == 8)
        hipLaunchKernelGGL(conv_fwd_kernel<8>, grid, dim3(c.threads), lds, st, x, w, bias, y, Ci, Co, in[0], in[1],
                           in[2], out[0], out[1], out[2], s, act);
    else
        hipLaunchKernelGGL(conv_fwd_kernel<4>, grid, dim3(c.threads), lds, st, x, w, bias, y, Ci, Co, in[0], in[1],
                           in[2], out[0], out[1], out[2], s, act);
    HIP_OK(hipGetLastError());
}

void conv_bwd_data(const float* gout, const uint16_t* w, float* gin, int B, int Ci, int Co, const int in[3],
                   const int out[3], int s, int accumulate, hipStream_t st) {
    const int nv = in[0] * in[1] * in[2];
    const ConvShape c = conv_shape((int64_t)B * nv, Co * 27);
    const size_t lds = (size_t)c.tile * Co * 27 * sizeof(float);
    dim3 grid(grid1(nv, c.threads), (unsigned)((Ci + c.tile - 1) / c.tile), (unsigned)B);
    if (c.tile == 16)
        hipLaunchKernelGGL(conv_bwd_data_kernel<16>, grid, dim3(c.threads), lds, st, gout, w, gin, Ci, Co, in[0],
                           in[1], in[2], out[0], out[1], out[2], s, accumulate);
    else if (c.tile == 8)
        hipLaunchKernelGGL(conv_bwd_data_kernel<8>, grid, dim3(c.threads), lds, st, gout, w, gin, Ci, Co, in[0],
                           in[1], in[2], out[0], out[1], out[2], s, accumulate);
    else
        hipLaunchKernelGGL(conv_bwd_data_kernel<4>, grid, dim3(c.threads), lds, st, gout, w, gin, Ci, Co, in[0],
                           in[1], in[2], out[0], out[1], out[2], s, accumulate);
    HIP_OK(hipGetLastError());
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
    uint16_t* wbf = nullptr;     // BF16 copy used by the convolutions
    int64_t adam_t = 0;
    // workspace for the current shape
    int B = 0, dims[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    std::vector<float*> act;     // T_COUNT activations
    std::vector<float*> gact;    // their gradients
    float* gx_tmp = nullptr;     // gradient of the input when not requested
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
}

// conv layer k: input tensor (or x), output tensor
struct Wiring {
    int in, out;   // tensor ids (-1 = network input)
};
const Wiring kWire[12] = {{-1, T_E0A}, {T_E0A, T_S0}, {T_S0, T_E1A}, {T_E1A, T_S1}, {T_S1, T_E2A}, {T_E2A, T_E2B},
                          {T_E2B, T_E2C}, {T_E2C, T_U1A}, {T_H1, T_U1B}, {T_U1B, T_U0A}, {T_H0, T_U0B}, {T_U0B, T_Y}};

void run_conv(snsw_net* net, int k, const float* x, hipStream_t s) {
    const NetLayer& L = net->layers[k];
    const float* in = kWire[k].in < 0 ? x : net->act[kWire[k].in];
    const int lin = L.level_in, lout = L.stride == 2 ? lin + 1 : lin;
    conv_fwd(in, net->wbf + L.w_off, net->theta + L.b_off, net->act[kWire[k].out], net->B, L.cin, L.cout,
             net->dims[lin], net->dims[lout], L.stride, L.act, s);
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
    hipLaunchKernelGGL(conv_bwd_weight_kernel, dim3((unsigned)(L.cout * L.cin)), dim3(256), 0, s, in, gout,
                       net->grad + L.w_off, net->B, L.cin, L.cout, di[0], di[1], di[2], dout[0], dout[1], dout[2],
                       L.stride);
    HIP_OK(hipGetLastError());
    hipLaunchKernelGGL(bias_grad_kernel, dim3((unsigned)L.cout), dim3(256), 0, s, gout, net->grad + L.b_off, net->B,
                       L.cout, dout[0] * dout[1] * dout[2]);
    HIP_OK(hipGetLastError());
    if (gin) conv_bwd_data(gout, net->wbf + L.w_off, gin, net->B, L.cin, L.cout, di, dout, L.stride, accumulate, s);
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
    void* ptrs[] = {net->theta, net->m, net->v, net->grad, net->wbf, net->loss_dev,
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
        HIP_OK(hipMalloc(&net->loss_dev, sizeof(double)));
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
        hipLaunchKernelGGL(mse_kernel, dim3(1), dim3(1024), 0, s, d_y, d_t, count, d_dy, net->loss_dev);
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
