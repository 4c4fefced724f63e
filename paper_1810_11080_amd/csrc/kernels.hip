// HIP kernels of the lagged transport sweep for gfx950.
//
// One launch processes every (element, direction) pair of one level of the
// combined schedule: their upwind inputs were produced by earlier levels
// (kept couplings) or by the previous sweep (lagged couplings), so all pairs
// of a level are independent.  Per pair the local system of eq.
// laggedSourceIteration is assembled and solved in registers:
//
//   A = sigma_t M - sum_i Omega_i K_i + sum_{outflow faces} P_out
//   b = M (q + sigma_s/(4 pi) phi) + sum_{inflow faces} P_in psi_upwind
//
// Mapping: a wavefront holds G = 64 / n pairs, lane `row` of a group owns row
// `row` of A and b.  Elimination without pivoting (the symmetric part of A is
// positive definite: A + A^T = 2 sigma_t M + int |Omega.n| u u over the
// element boundary) broadcasts the pivot row through LDS.  Matrices are read
// column-major so that the n lanes of a group load consecutive addresses.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace snsw {

namespace {

constexpr int kWaves = 4;              // wavefronts per block
constexpr int kDirMask = 1023;         // packed word: direction bits
constexpr int kSlotShift = 10;         // then 3 bits per slot
constexpr unsigned kOut = 0, kIn = 1, kKink = 2;

template <int DIM, int P>
struct Shape {
    static constexpr int Q = P + 1;
    static constexpr int N = DIM == 2 ? Q * Q : Q * Q * Q;
    static constexpr int NF = DIM == 2 ? Q : Q * Q;
    static constexpr int NS = 2 * DIM;
    static constexpr int G = 64 / N;
    __host__ __device__ static constexpr int coord(int i, int a) {
        return a == 0 ? i % Q : (a == 1 ? (i / Q) % Q : i / (Q * Q));
    }
    // element node of face-local index b on slot s (remaining axes ascending)
    __host__ __device__ static constexpr int tn(int s, int b) {
        int idx[3] = {0, 0, 0};
        int rem = b;
        for (int x = 0; x < DIM; ++x) {
            if (x == s / 2) continue;
            idx[x] = rem % Q;
            rem /= Q;
        }
        idx[s / 2] = (s & 1) ? P : 0;
        return idx[0] + Q * (idx[1] + Q * idx[2]);
    }
    // face-local index of node i on slot s
    __host__ __device__ static constexpr int local(int i, int s) {
        int l = 0, mul = 1;
        for (int x = 0; x < DIM; ++x) {
            if (x == s / 2) continue;
            l += coord(i, x) * mul;
            mul *= Q;
        }
        return l;
    }
};

template <int DIM, int P>
__global__ void __launch_bounds__(64 * kWaves) sweep_level_fp64(SweepArgs args, int64_t begin, int64_t count) {
    using S = Shape<DIM, P>;
    constexpr int N = S::N, NF = S::NF, NS = S::NS, G = S::G;
    __shared__ double lds[kWaves][G][N + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int grp = lane / N, row = lane - grp * N;
    const bool in_group = grp < G;
    const int64_t pidx = begin + ((int64_t)blockIdx.x * kWaves + wave) * G + grp;
    const bool active = in_group && pidx < begin + count;

    double a[N];
    double rhs = 0.0;
    int e = 0, d = 0;
    if (active) {
        const int4 pr = args.pairs[pidx];
        e = pr.x;
        const unsigned packed = (unsigned)pr.y;
        const int kb = pr.z;
        d = (int)(packed & kDirMask);
        const double* Ge = args.geo + (size_t)e * (DIM + 1) * N * N;
        const double st = args.sigma_t[e];
        const double o0 = args.omega[3 * d + 0], o1 = args.omega[3 * d + 1], o2 = args.omega[3 * d + 2];
#pragma unroll
        for (int j = 0; j < N; ++j) {
            double v = st * Ge[j * N + row];
            v -= o0 * Ge[1 * N * N + j * N + row];
            v -= o1 * Ge[2 * N * N + j * N + row];
            if (DIM == 3) v -= o2 * Ge[3 * N * N + j * N + row];
            a[j] = v;
        }
        rhs = args.src[(size_t)e * N + row];
        int kc = 0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const unsigned cls = (packed >> (kSlotShift + 3 * s)) & 3u;
            const bool lagged = (packed >> (kSlotShift + 3 * s + 2)) & 1u;
            int krow = 0;
            if (cls == kKink) krow = args.kink_idx[kb + kc++];
            const bool on = S::coord(row, s / 2) == ((s & 1) ? P : 0);
            if (!on) continue;
            const int la = S::local(row, s);
            double pout[NF], pin[NF];
            if (cls == kKink) {
                // element is the face's minus side on odd slots: out = P_plus
                const double* T = args.kink_tab + (size_t)krow * 2 * NF * NF;
                const double* To = T + ((s & 1) ? 0 : NF * NF);
                const double* Ti = T + ((s & 1) ? NF * NF : 0);
#pragma unroll
                for (int b = 0; b < NF; ++b) {
                    pout[b] = To[la * NF + b];
                    pin[b] = Ti[la * NF + b];
                }
            } else {
                const int f = args.slot_face[(size_t)e * NS + s];
                const double* Bf = args.B + (size_t)f * DIM * NF * NF + la * NF;
                const double sgn = (s & 1) ? 1.0 : -1.0;   // outward normal = sgn * N
#pragma unroll
                for (int b = 0; b < NF; ++b) {
                    double v = o0 * Bf[b] + o1 * Bf[NF * NF + b];
                    if (DIM == 3) v += o2 * Bf[2 * NF * NF + b];
                    v *= sgn;                               // int (Omega . n_out) phi phi
                    pout[b] = cls == kOut ? v : 0.0;
                    pin[b] = cls == kOut ? 0.0 : -v;
                }
            }
#pragma unroll
            for (int b = 0; b < NF; ++b) a[S::tn(s, b)] += pout[b];
            if (cls != kOut) {
                const int nb = args.slot_nbr[(size_t)e * NS + s];
                if (nb >= 0) {
                    const double* up = (lagged ? args.psi_prev : args.psi_cur) + ((size_t)d * args.E + nb) * N;
#pragma unroll
                    for (int b = 0; b < NF; ++b) rhs += pin[b] * up[S::tn(s ^ 1, b)];
                } else {
#pragma unroll
                    for (int b = 0; b < NF; ++b) rhs += pin[b] * args.psi_inc;
                }
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < N; ++j) a[j] = (j == row) ? 1.0 : 0.0;
    }

    // Gaussian elimination, pivot row broadcast through LDS
#pragma unroll
    for (int k = 0; k < N; ++k) {
        if (in_group && row == k) {
#pragma unroll
            for (int j = k; j < N; ++j) lds[wave][grp][j] = a[j];
            lds[wave][grp][N] = rhs;
        }
        __syncthreads();
        if (in_group && row > k) {
            const double l = a[k] / lds[wave][grp][k];
#pragma unroll
            for (int j = k + 1; j < N; ++j) a[j] -= l * lds[wave][grp][j];
            rhs -= l * lds[wave][grp][N];
        }
        __syncthreads();
    }
    // back substitution
    double x = 0.0;
#pragma unroll
    for (int k = N - 1; k >= 0; --k) {
        if (in_group && row == k) {
            x = rhs / a[k];
            lds[wave][grp][0] = x;
        }
        __syncthreads();
        if (in_group && row < k) rhs -= a[k] * lds[wave][grp][0];
        __syncthreads();
    }
    if (active) args.psi_cur[((size_t)d * args.E + e) * N + row] = x;
}

template <int DIM, int P>
void launch_tpl(const SweepArgs& a, int64_t begin, int64_t count, hipStream_t stream) {
    constexpr int per_block = kWaves * Shape<DIM, P>::G;
    const int64_t blocks = (count + per_block - 1) / per_block;
    if (blocks == 0) return;
    hipLaunchKernelGGL((sweep_level_fp64<DIM, P>), dim3((unsigned)blocks), dim3(64 * kWaves), 0, stream, a,
                       begin, count);
}

__global__ void source_kernel(int dim, int n, int64_t E, const double* __restrict__ geo,
                              const double* __restrict__ q, const double* __restrict__ sigma_s,
                              const double* __restrict__ phi, double* __restrict__ src) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= E * n) return;
    const int64_t e = t / n;
    const int i = (int)(t - e * n);
    const double c = sigma_s[e] * (0.25 / M_PI);
    const double* M = geo + (size_t)e * (dim + 1) * n * n;
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += M[(size_t)j * n + i] * (q[e * n + j] + c * phi[e * n + j]);
    src[t] = s;
}

__global__ void scalar_flux_kernel(int D, int64_t En, const double* __restrict__ w,
                                   const double* __restrict__ psi, double* __restrict__ phi) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= En) return;
    double s = 0.0;
    for (int d = 0; d < D; ++d) s += w[d] * psi[(size_t)d * En + t];
    phi[t] = s;
}

__global__ void residual_kernel(int64_t len, const double* __restrict__ a, const double* __restrict__ b,
                                unsigned long long* out) {
    __shared__ double s0[256], s1[256];
    double m0 = 0.0, m1 = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < len; t += (int64_t)gridDim.x * blockDim.x) {
        const double x = a[t], y = b[t];
        const double dd = fabs(x - y), ax = fabs(x);
        m0 = (dd > m0 || dd != dd) ? dd : m0;   // keeps a NaN
        m1 = (ax > m1 || ax != ax) ? ax : m1;
    }
    s0[threadIdx.x] = m0;
    s1[threadIdx.x] = m1;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            const double u0 = s0[threadIdx.x + st], u1 = s1[threadIdx.x + st];
            if (u0 > s0[threadIdx.x] || u0 != u0) s0[threadIdx.x] = u0;
            if (u1 > s1[threadIdx.x] || u1 != u1) s1[threadIdx.x] = u1;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        // nonnegative doubles order like their bit patterns; NaN sorts last
        atomicMax(&out[0], (unsigned long long)__double_as_longlong(s0[0]));
        atomicMax(&out[1], (unsigned long long)__double_as_longlong(s1[0]));
    }
}

}  // namespace

void launch_sweep_level(int dim, int p, bool mixed, const SweepArgs& a, int64_t begin, int64_t count,
                        hipStream_t stream) {
    (void)mixed;
    if (dim == 2) {
        if (p == 1) launch_tpl<2, 1>(a, begin, count, stream);
        else if (p == 2) launch_tpl<2, 2>(a, begin, count, stream);
        else launch_tpl<2, 3>(a, begin, count, stream);
    } else {
        if (p == 1) launch_tpl<3, 1>(a, begin, count, stream);
        else if (p == 2) launch_tpl<3, 2>(a, begin, count, stream);
        else launch_tpl<3, 3>(a, begin, count, stream);
    }
}

void launch_source(int dim, int n, int64_t E, const double* geo, const double* q, const double* sigma_s,
                   const double* phi, double* src, hipStream_t stream) {
    const int64_t tot = E * n;
    const int64_t blocks = (tot + 255) / 256;
    hipLaunchKernelGGL(source_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, dim, n, E, geo, q, sigma_s,
                       phi, src);
}

void launch_scalar_flux(int D, int64_t En, const double* w, const double* psi, double* phi, hipStream_t stream) {
    const int64_t blocks = (En + 255) / 256;
    hipLaunchKernelGGL(scalar_flux_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, D, En, w, psi, phi);
}

void launch_residual(int64_t len, const double* a, const double* b, unsigned long long* out, hipStream_t stream) {
    int64_t blocks = (len + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(residual_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, len, a, b, out);
}

}  // namespace snsw
