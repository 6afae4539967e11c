// HIP kernels of the Synch-EM iteration for gfx950 (CDNA4, wave64).
//
// One EM iteration (Algorithm "Synch-EM"; Section II-B eqs. (15), (17), (18); App. C eq. (42)):
//   template_kernel  T[:, i] = a_t o exp(-i kbar theta_{o_i}), written in MFMA B-fragment order
//   pass_kernel      per row tile: C = [Re V, Im V] [Re T; Im T] on matrix cores, then
//                    l_ji = 2 C_ji / sigma^2 + log rho_i, per-row log-sum-exp, posteriors,
//                    U_jk = sum_i w_ji exp(+i k theta_i), S_d += sum_j U_{j,kbar_d} v_jd,
//                    W_i += sum_j w_ji; FP64 per-workgroup partials
//   reduce_kernel    fixed-order FP64 sum of the partials (set-up sums)
//   reduce_finalize_kernel  the same sum of a pass's partials, more workgroups per column; the
//                    workgroup that finishes last then computes, in FP64, a_{t+1}, rho_{t+1}, the
//                    log-likelihood, the MAP objective and the stopping metric
//
// The per-row constants -(||v_j||^2 + ||a||^2)/sigma^2 - D log(pi sigma^2) of the log-weights are
// left out of the pass (they cancel in the posteriors) and added back in FP64 in the finalize.
#include "em_internal.h"

#include <hip/hip_ext.h>
#include <math.h>
#include <stdio.h>

#include <type_traits>

namespace sem {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------------------------------
// small helpers

__device__ __forceinline__ float bf16_to_f(__bf16 x) { return (float)x; }
__device__ __forceinline__ float f16_to_f(_Float16 x) { return (float)x; }

template <typename T>
__device__ __forceinline__ T group_max(T v, int width) {
    for (int o = width >> 1; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, width));
    return v;
}
template <typename T>
__device__ __forceinline__ T group_sum(T v, int width) {
    for (int o = width >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, width);
    return v;
}

// Workgroup barrier for LDS hand-offs only: waits for this wave's LDS accesses, not for its
// vector-memory loads (a __syncthreads() would also drain the copies and prefetch loads still in
// flight, which every pass keeps in flight across its tile phases).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_s_waitcnt(15 | (7 << 4) | (0 << 8) | (3 << 14));
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// Deterministic block sum of one double per thread (fixed tree order). All threads get the sum.
__device__ double block_sum_d(double v, double *sh, int n) {
    const int t = threadIdx.x;
    __syncthreads();
    sh[t] = v;
    __syncthreads();
    for (int s = n >> 1; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}
__device__ double block_min_d(double v, double *sh, int n) {
    const int t = threadIdx.x;
    __syncthreads();
    sh[t] = v;
    __syncthreads();
    for (int s = n >> 1; s > 0; s >>= 1) {
        if (t < s) sh[t] = fmin(sh[t], sh[t + s]);
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// Storage scaling: observations and template are multiplied by a power of two before rounding
// to 16-bit so that the largest magnitude lands in [2^E, 2^(E+1)); fp16 uses E = 14 (the top of
// its range keeps small entries out of the subnormals), bf16 E = 0.  FP32/FP64 are not scaled.
__host__ __device__ __forceinline__ int scale_target(int prec) {
    return prec == P_F16 ? 14 : 0;
}
__device__ __forceinline__ bool prec_scaled(int prec) {
    return prec == P_BF16X3 || prec == P_F16 || prec == P_BF16;
}

// ------------------------------------------------------------------------------------------
// a1: observation conversion (once, at init).  One wave per row.

template <int P>
__global__ __launch_bounds__(256) void convert_kernel(const void *obs, int64_t N, int D, int Dp,
                                                      uint8_t *V, int64_t rowbytes,
                                                      float *rowscale, double *vnorm2,
                                                      int *nonfinite) {
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * 4;
    for (int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); row < N; row += waves) {
        double n2 = 0.0;
        float amax = 0.0f;
        bool bad = false;
        for (int d = lane; d < D; d += 64) {
            double re, im;
            if (P == P_F64) {
                const double2 v = ((const double2 *)obs)[row * D + d];
                re = v.x;
                im = v.y;
            } else {
                const float2 v = ((const float2 *)obs)[row * D + d];
                re = v.x;
                im = v.y;
            }
            bad |= !isfinite(re) || !isfinite(im);
            n2 += re * re + im * im;
            amax = fmaxf(amax, fmaxf(fabsf((float)re), fabsf((float)im)));
        }
        n2 = group_sum(n2, 64);
        amax = group_max(amax, 64);
        if (bad) atomicOr(nonfinite, 1);
        float sc = 1.0f, unsc = 1.0f;
        if (prec_scaled(P) && amax > 0.0f && isfinite(amax)) {
            const int e = ilogbf(amax);
            sc = ldexpf(1.0f, scale_target(P) - e);
            unsc = ldexpf(1.0f, e - scale_target(P));
        }
        if (lane == 0) {
            vnorm2[row] = n2;
            if (rowscale) rowscale[row] = unsc;
        }
        uint8_t *dst = V + row * rowbytes;
        for (int d = lane; d < Dp / 2; d += 64) {
            float re = 0.f, im = 0.f;
            double dre = 0.0, dim = 0.0;
            if (d < D) {
                if (P == P_F64) {
                    const double2 v = ((const double2 *)obs)[row * D + d];
                    dre = v.x;
                    dim = v.y;
                } else {
                    const float2 v = ((const float2 *)obs)[row * D + d];
                    re = v.x * sc;
                    im = v.y * sc;
                }
            }
            if (P == P_F64) {
                ((double2 *)dst)[d] = make_double2(dre, dim);
            } else if (P == P_F32) {
                ((float2 *)dst)[d] = make_float2(re, im);
            } else if (P == P_F16) {
                _Float16 *h = (_Float16 *)dst;
                h[2 * d] = (_Float16)re;
                h[2 * d + 1] = (_Float16)im;
            } else if (P == P_BF16) {
                __bf16 *h = (__bf16 *)dst;
                h[2 * d] = (__bf16)re;
                h[2 * d + 1] = (__bf16)im;
            } else {  // P_BF16X3: hi plane, then lo plane = x - hi (exact in fp32)
                __bf16 *h = (__bf16 *)dst;
                __bf16 *l = h + Dp;
                const __bf16 hr = (__bf16)re, hi_ = (__bf16)im;
                h[2 * d] = hr;
                h[2 * d + 1] = hi_;
                l[2 * d] = (__bf16)(re - (float)hr);
                l[2 * d + 1] = (__bf16)(im - (float)hi_);
            }
        }
    }
}

// Column sums of the observations (for the initial estimate a_0 = mean v), FP64 partials.
__global__ __launch_bounds__(512) void colsum_kernel(const void *obs, int is_c128, int64_t N,
                                                     int D, double *partials) {
    const int64_t rpb = (N + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * rpb;
    const int64_t r1 = r0 + rpb < N ? r0 + rpb : N;
    // eight rows in flight per thread (eight running sums, added in a fixed order at the end)
    for (int r = threadIdx.x; r < 2 * D; r += blockDim.x) {
        double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        int64_t j = r0;
        for (; j + 8 <= r1; j += 8) {
#pragma unroll
            for (int u = 0; u < 8; ++u)
                s[u] += is_c128 ? ((const double *)obs)[(j + u) * 2 * D + r]
                                : (double)((const float *)obs)[(j + u) * 2 * D + r];
        }
        for (int u = 0; j < r1; ++j, ++u)
            s[u] += is_c128 ? ((const double *)obs)[j * 2 * D + r]
                            : (double)((const float *)obs)[j * 2 * D + r];
        partials[(int64_t)blockIdx.x * 2 * D + r] =
            ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
    }
}

// Fixed-order FP64 sum of n values in two stages: workgroup b sums the contiguous range
// [b n / G, (b + 1) n / G) (eight strided running sums per thread, then a tree over the block)
// into partials[b]; sum_kernel2 adds the G partials in a fixed order.
__global__ __launch_bounds__(256) void sum_kernel(const double *x, int64_t n, double *partials) {
    __shared__ double sh[256];
    const int64_t b0 = n * blockIdx.x / gridDim.x, b1 = n * (blockIdx.x + 1) / gridDim.x;
    double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int64_t i = b0 + threadIdx.x;
    for (; i + 7 * 256 < b1; i += 8 * 256) {
#pragma unroll
        for (int u = 0; u < 8; ++u) s[u] += x[i + u * 256];
    }
    for (int u = 0; i < b1; i += 256, ++u) s[u] += x[i];
    double v = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = sh[0];
}
// One wave: lane l adds partials l, l + 64, ... in order, then a butterfly over the wave.
__global__ __launch_bounds__(64) void sum_kernel2(const double *partials, int G, double *out) {
    const int l = threadIdx.x;
    double t = 0.0;
    for (int b = l; b < G; b += 64) t += partials[b];
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) t += __shfl_xor(t, m, 64);
    if (l == 0) *out = t;
}

// Fixed-order FP64 reduction over workgroup partials: out[c] = sum_b partials[b][c].
__global__ __launch_bounds__(512) void reduce_kernel(const double *partials, int G, int ncols,
                                                     double *out) {
    __shared__ double sh[8][64];
    const int cl = threadIdx.x & 63, gs = threadIdx.x >> 6;
    const int col = blockIdx.x * 64 + cl;
    double s = 0.0;
    if (col < ncols) {
#pragma unroll 8
        for (int b = gs; b < G; b += 8) s += partials[(int64_t)b * ncols + col];
    }
    sh[gs][cl] = s;
    __syncthreads();
    if (gs == 0 && col < ncols) {
        double t = 0.0;
        for (int k = 0; k < 8; ++k) t += sh[k][cl];
        out[col] = t;
    }
}

__global__ void scale_kernel(const double *in, double *out, int n, double f) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[i] * f;
}

// log rho into the padded FP32/FP64 buffers (-inf on zero entries and on the padding).
__device__ void write_logrho(const double *rho, float *l32, double *l64, int W, int Wp) {
    for (int i = threadIdx.x; i < Wp; i += blockDim.x) {
        const double r = i < W ? rho[i] : 0.0;
        const double l = r > 0.0 ? log(r) : -INFINITY;
        l32[i] = (float)l;
        l64[i] = l;
    }
}

__global__ void logrho_kernel(const double *rho, float *l32, double *l64, int W, int Wp) {
    write_logrho(rho, l32, l64, W, Wp);
}

// rho = softmax(eta) over the window (one workgroup of 256), then its log.
__global__ __launch_bounds__(256) void softmax_kernel(const double *eta, double *rho, float *l32,
                                                      double *l64, int W, int Wp) {
    __shared__ double sh[256];
    double m = -INFINITY;
    for (int i = threadIdx.x; i < W; i += 256) m = fmax(m, eta[i]);
    m = -block_min_d(-m, sh, 256);
    double s = 0.0;
    for (int i = threadIdx.x; i < W; i += 256) s += exp(eta[i] - m);
    s = block_sum_d(s, sh, 256);
    for (int i = threadIdx.x; i < W; i += 256) rho[i] = exp(eta[i] - m) / s;
    __syncthreads();
    write_logrho(rho, l32, l64, W, Wp);
}

// ------------------------------------------------------------------------------------------
// a2: template T[r][i] (r: real index 2d / 2d+1 = Re / Im of entry d; i: window column), with
// T[., i] = a o exp(-i kbar theta_{o_i}) evaluated at the exact grid angle 2 pi ((k o_i) mod L)/L.
// Stored in MFMA B-fragment order so a lane's operand is one 16-byte load:
//   FP32  (16x16x4):  [nt][r/16][lane][4],  lane = 16*((r%16)/4) + i%16, elem = r%4
//   16-bit(16x16x32): [nt][r/32][lane][8],  lane = 16*((r%32)/8) + i%16, elem = r%8
//   FP64  (VALU):     [r][Wp]
// nt = i/16.  The A operand (observation rows in LDS) is read with the same k order.

__global__ __launch_bounds__(256) void template_kernel(TplArgs A) {
    if (A.stopped && *A.stopped) return;
    __shared__ double sh[256];
    double amax = 0.0;
    for (int r = threadIdx.x; r < 2 * A.D; r += 256) amax = fmax(amax, fabs(A.a[r]));
    amax = -block_min_d(-amax, sh, 256);
    double sc = 1.0;
    float unsc = 1.0f;
    if ((A.prec == P_BF16X3 || A.prec == P_F16 || A.prec == P_BF16) && amax > 0.0) {
        const int e = ilogb(amax);
        sc = ldexp(1.0, scale_target(A.prec) - e);
        unsc = ldexpf(1.0f, e - scale_target(A.prec));
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *A.tscale = unsc;

    const int half = A.Dp / 2;
    const int64_t total = (int64_t)half * A.Wp;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < total;
         p += (int64_t)gridDim.x * 256) {
        const int d = (int)(p / A.Wp);
        const int i = (int)(p - (int64_t)d * A.Wp);
        double tre = 0.0, tim = 0.0;
        if (d < A.D && i < A.W) {
            const int k = d / A.Q;
            const double2 ph = A.E64[(int64_t)i * A.K + k];   // exp(+i k theta_i)
            const double are = A.a[2 * d], aim = A.a[2 * d + 1];
            tre = (are * ph.x + aim * ph.y) * sc;      // a * conj(ph)
            tim = (aim * ph.x - are * ph.y) * sc;
        }
        const int r = 2 * d;
        const int nt = i >> 4, col = i & 15;
        if (A.prec == P_F64) {
            double *T = (double *)A.Thi;
            T[(int64_t)r * A.Wp + i] = tre;
            T[(int64_t)(r + 1) * A.Wp + i] = tim;
        } else if (A.prec == P_F32) {
            const int KG = A.Dp / 16, kg = r >> 4, w = r & 15;
            const int lane = 16 * (w >> 2) + col;
            float *T = (float *)A.Thi + (((int64_t)nt * KG + kg) * 64 + lane) * 4 + (w & 3);
            T[0] = (float)tre;
            T[1] = (float)tim;
        } else {
            const int KS = A.Dp / 32, ks = r >> 5, w = r & 31;
            const int lane = 16 * (w >> 3) + col;
            const int64_t off = (((int64_t)nt * KS + ks) * 64 + lane) * 8 + (w & 7);
            if (A.prec == P_F16) {
                _Float16 *H = (_Float16 *)A.Thi + off, *Lo = (_Float16 *)A.Tlo + off;
                const _Float16 hr = (_Float16)tre, hi_ = (_Float16)tim;
                H[0] = hr;
                H[1] = hi_;
                Lo[0] = (_Float16)(tre - (double)(float)hr);
                Lo[1] = (_Float16)(tim - (double)(float)hi_);
            } else {
                __bf16 *H = (__bf16 *)A.Thi + off, *Lo = (__bf16 *)A.Tlo + off;
                const __bf16 hr = (__bf16)(float)tre, hi_ = (__bf16)(float)tim;
                H[0] = hr;
                H[1] = hi_;
                Lo[0] = (__bf16)(float)(tre - (double)(float)hr);
                Lo[1] = (__bf16)(float)(tim - (double)(float)hi_);
            }
        }
    }
}

// ------------------------------------------------------------------------------------------
// a3-a5: the fused E(+M) pass.

template <int P> struct PT {                      // compute type of the epilogue
    typedef float CT;
    typedef float2 CT2;
};
template <> struct PT<P_F64> {
    typedef double CT;
    typedef double2 CT2;
};

__host__ __device__ constexpr int align_up(int x, int a) { return (x + a - 1) / a * a; }

// LDS layout of the pass: [V tile(s): nbuf x BM x RS bytes][C tile: BM x CSW][U tile: BM x K]
// [row factors: BM x 2].  nbuf = 2 when the tile is double-buffered by direct global-to-LDS
// copies.
struct PassLds {
    int RS, CSW;
    int off_v1, off_c, off_u, off_f, off_lr, total;
};
__host__ __device__ inline PassLds pass_lds(int prec, int BM, int K, int Dp, int Wp, int nbuf) {
    PassLds l;
    const int rb = (int)row_bytes(prec, Dp);
    const int cs = prec == P_F64 ? 8 : 4;
    l.RS = rb + 16;
    l.CSW = Wp + 1;
    l.off_v1 = align_up(BM * l.RS, 16);
    l.off_c = align_up(nbuf * BM * l.RS, 16);
    l.off_u = align_up(l.off_c + BM * l.CSW * cs, 16);
    l.off_f = align_up(l.off_u + BM * K * 2 * cs, 16);
    l.off_lr = align_up(l.off_f + 2 * BM * cs, 16);
    l.total = l.off_lr + Wp * 4 + 16;
    return l;
}

// Complex entry d of a stored row, as the compute type (still in the row's storage scale).
template <int P>
__device__ __forceinline__ typename PT<P>::CT2 load_v(const uint8_t *row, int d, int Dp) {
    if constexpr (P == P_F64) {
        return *(const double2 *)(row + 16 * d);
    } else if constexpr (P == P_F32) {
        return *(const float2 *)(row + 8 * d);
    } else if constexpr (P == P_F16) {
        const _Float16 *h = (const _Float16 *)(row + 4 * d);
        return make_float2((float)h[0], (float)h[1]);
    } else if constexpr (P == P_BF16) {
        const __bf16 *h = (const __bf16 *)(row + 4 * d);
        return make_float2((float)h[0], (float)h[1]);
    } else {
        const __bf16 *h = (const __bf16 *)(row + 4 * d);
        const __bf16 *l = (const __bf16 *)(row + 2 * Dp + 4 * d);
        return make_float2((float)h[0] + (float)l[0], (float)h[1] + (float)l[1]);
    }
}

// The same entry read as whole 32-bit words (bf16 widened by a shift): for the M-step loops.
template <int P>
__device__ __forceinline__ float2 load_v32(const uint8_t *row, int d, int Dp) {
    if constexpr (P == P_F32) {
        return *(const float2 *)(row + 8 * d);
    } else if constexpr (P == P_F16) {
        const uint32_t w = *(const uint32_t *)(row + 4 * d);
        const _Float16 *h = (const _Float16 *)&w;
        return make_float2((float)h[0], (float)h[1]);
    } else {
        const uint32_t w = *(const uint32_t *)(row + 4 * d);
        float re = __uint_as_float(w << 16), im = __uint_as_float(w & 0xffff0000u);
        if constexpr (P == P_BF16X3) {
            const uint32_t l = *(const uint32_t *)(row + 2 * Dp + 4 * d);
            re += __uint_as_float(l << 16);
            im += __uint_as_float(l & 0xffff0000u);
        }
        return make_float2(re, im);
    }
}

// Correlations of MSW 16-row blocks (rows (wm + m WM) 16 ..) with up to NTW 16-column tiles
// (nt0, nt0 + WN, ...) of the template, MFMA paths.  A fragments come from the LDS tile, B
// fragments stream from L2 through a ring of PD k-steps in registers.
template <int P, int MSW, int WM, int NTW, int PD>
__device__ __forceinline__ void gemm_ntiles(f32x4 (&acc)[NTW][MSW], const uint8_t *Vs, int RS,
                                            int wm, int lane, int nt0, int WN, int NT, int Dp,
                                            const void *Thi, const void *Tlo) {
    const int g = lane >> 4, rl = lane & 15;
    bool ok[NTW];
#pragma unroll
    for (int n = 0; n < NTW; ++n) {
        ok[n] = nt0 + n * WN < NT;
#pragma unroll
        for (int m = 0; m < MSW; ++m) acc[n][m] = (f32x4){0.f, 0.f, 0.f, 0.f};
    }
    const uint8_t *Arow[MSW];
#pragma unroll
    for (int m = 0; m < MSW; ++m) Arow[m] = Vs + ((wm + m * WM) * 16 + rl) * RS + g * 16;
    if constexpr (P == P_F32) {
        const int KG = Dp / 16;
        const float4 *B[NTW];
        float4 b[PD][NTW];
#pragma unroll
        for (int n = 0; n < NTW; ++n) B[n] = (const float4 *)Thi + (int64_t)(nt0 + n * WN) * KG * 64 + lane;
#pragma unroll
        for (int u = 0; u < PD; ++u)
#pragma unroll
            for (int n = 0; n < NTW; ++n)
                if (ok[n] && u < KG) b[u][n] = B[n][u * 64];
        for (int kg0 = 0; kg0 < KG; kg0 += PD) {
#pragma unroll
            for (int u = 0; u < PD; ++u) {
                const int kg = kg0 + u;
                if (kg >= KG) break;
                float4 a[MSW];
#pragma unroll
                for (int m = 0; m < MSW; ++m) a[m] = *(const float4 *)(Arow[m] + kg * 64);
#pragma unroll
                for (int n = 0; n < NTW; ++n) {
                    if (!ok[n]) continue;
                    const float4 bb = b[u][n];
#pragma unroll
                    for (int m = 0; m < MSW; ++m) {
                        acc[n][m] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[m].x, bb.x, acc[n][m], 0, 0, 0);
                        acc[n][m] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[m].y, bb.y, acc[n][m], 0, 0, 0);
                        acc[n][m] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[m].z, bb.z, acc[n][m], 0, 0, 0);
                        acc[n][m] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[m].w, bb.w, acc[n][m], 0, 0, 0);
                    }
                    if (kg + PD < KG) b[u][n] = B[n][(kg + PD) * 64];
                }
            }
        }
    } else {
        const int KS = Dp / 32;
        const u32x4 *Bh[NTW], *Bl[NTW];
        u32x4 bh[PD][NTW], bl[PD][NTW];
#pragma unroll
        for (int n = 0; n < NTW; ++n) {
            Bh[n] = (const u32x4 *)Thi + (int64_t)(nt0 + n * WN) * KS * 64 + lane;
            Bl[n] = (const u32x4 *)Tlo + (int64_t)(nt0 + n * WN) * KS * 64 + lane;
        }
#pragma unroll
        for (int u = 0; u < PD; ++u)
#pragma unroll
            for (int n = 0; n < NTW; ++n)
                if (ok[n] && u < KS) {
                    bh[u][n] = Bh[n][u * 64];
                    bl[u][n] = Bl[n][u * 64];
                }
        for (int ks0 = 0; ks0 < KS; ks0 += PD) {
#pragma unroll
            for (int u = 0; u < PD; ++u) {
                const int ks = ks0 + u;
                if (ks >= KS) break;
                u32x4 ah[MSW], al[MSW];
#pragma unroll
                for (int m = 0; m < MSW; ++m) {
                    ah[m] = *(const u32x4 *)(Arow[m] + ks * 64);
                    if constexpr (P == P_BF16X3) al[m] = *(const u32x4 *)(Arow[m] + 2 * Dp + ks * 64);
                }
#pragma unroll
                for (int n = 0; n < NTW; ++n) {
                    if (!ok[n]) continue;
                    const u32x4 BH = bh[u][n], BL = bl[u][n];
#pragma unroll
                    for (int m = 0; m < MSW; ++m) {
                        if constexpr (P == P_F16) {
                            const f16x8 A8 = __builtin_bit_cast(f16x8, ah[m]);
                            acc[n][m] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                                A8, __builtin_bit_cast(f16x8, BL), acc[n][m], 0, 0, 0);
                            acc[n][m] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                                A8, __builtin_bit_cast(f16x8, BH), acc[n][m], 0, 0, 0);
                        } else if constexpr (P == P_BF16) {
                            const bf16x8 A8 = __builtin_bit_cast(bf16x8, ah[m]);
                            acc[n][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                A8, __builtin_bit_cast(bf16x8, BL), acc[n][m], 0, 0, 0);
                            acc[n][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                A8, __builtin_bit_cast(bf16x8, BH), acc[n][m], 0, 0, 0);
                        } else {  // P_BF16X3
                            const bf16x8 AH = __builtin_bit_cast(bf16x8, ah[m]);
                            acc[n][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                AH, __builtin_bit_cast(bf16x8, BL), acc[n][m], 0, 0, 0);
                            acc[n][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                __builtin_bit_cast(bf16x8, al[m]), __builtin_bit_cast(bf16x8, BH),
                                acc[n][m], 0, 0, 0);
                            acc[n][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                AH, __builtin_bit_cast(bf16x8, BH), acc[n][m], 0, 0, 0);
                        }
                    }
                    if (ks + PD < KS) {
                        bh[u][n] = Bh[n][(ks + PD) * 64];
                        bl[u][n] = Bl[n][(ks + PD) * 64];
                    }
                }
            }
        }
    }
}

// Accumulators a workgroup carries across its tiles (FP64): S for DPT complex entries per thread,
// W_t for two window columns per thread, and the per-row sums of log-sum-exp, w*C and rows.
template <int DPT>
struct PassAcc {
    double2 S[DPT];
    double W[2];
    double lse, wc, rows;
    __device__ __forceinline__ void init() {
#pragma unroll
        for (int c = 0; c < DPT; ++c) S[c] = make_double2(0.0, 0.0);
        W[0] = W[1] = 0.0;
        lse = wc = rows = 0.0;
    }
};

// Register-staged copy of one row tile (a contiguous byte range of the stored observations) into
// the LDS tile with padded rows.  issue() starts the loads; store() writes them to LDS.
template <int NPF>
struct TileLoader {
    u32x4 pf[NPF];
    __device__ __forceinline__ void issue(const PassArgs &A, int64_t tile, int BM) {
        const int tid = threadIdx.x;
        const int64_t r0 = A.row_begin + tile * BM;
        const int64_t rows = (A.row_end - r0) < BM ? (A.row_end - r0) : BM;
        const int64_t nbytes = rows * A.rowbytes;
        const u32x4 *src = (const u32x4 *)(A.V + r0 * A.rowbytes);
#pragma unroll
        for (int c = 0; c < NPF; ++c) {
            const int64_t ch = (int64_t)c * kThreads + tid;
            pf[c] = (ch * 16 < nbytes) ? src[ch] : (u32x4){0u, 0u, 0u, 0u};
        }
    }
    __device__ __forceinline__ void store(uint8_t *Vs, int RS, int BM, int64_t rowbytes) {
        const int tid = threadIdx.x;
        const int64_t tbytes = (int64_t)BM * rowbytes;
#pragma unroll
        for (int c = 0; c < NPF; ++c) {
            const int64_t ch = (int64_t)c * kThreads + tid;
            if (ch * 16 < tbytes) {
                const int byte = (int)(ch * 16);
                const int r = byte / (int)rowbytes;
                const int off = byte - r * (int)rowbytes;
                *(u32x4 *)(Vs + r * RS + off) = pf[c];
            }
        }
    }
};

// U (BM x 2K, as complex [BM][K]) = w (BM x Wp, the posterior tile in LDS) . [Re E | Im E]
// (Wp x 2K) on FP32 matrix cores (16x16x4), each row scaled by rowu; wave w computes the 16-column
// tiles w, w + 8, ... of U for all rows.  The B fragments stream from L2 through a RING-deep register ring.
template <int BM, int RING = 4>
__device__ __forceinline__ void u_mfma(const float *Cs, int CSW, const float *E2, int Wp, int K,
                                       const float *rowu, float2 *Us) {
    constexpr int MS = BM / 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, rl = lane & 15;
    const int NTU = (2 * K + 15) / 16, KG = Wp / 4;
    for (int nt = wave; nt < NTU; nt += kThreads / 64) {
        f32x4 acc[MS];
#pragma unroll
        for (int m = 0; m < MS; ++m) acc[m] = (f32x4){0.f, 0.f, 0.f, 0.f};
        const int col = nt * 16 + rl;
        const bool cok = col < 2 * K;
        const float *eb = E2 + (int64_t)g * 2 * K + (cok ? col : 0);
        float bq[RING];
#pragma unroll
        for (int u = 0; u < RING; ++u) bq[u] = (cok && u < KG) ? eb[(int64_t)u * 8 * K] : 0.f;
        for (int k0 = 0; k0 < KG; k0 += RING) {
#pragma unroll
            for (int u = 0; u < RING; ++u) {
                const int kk = k0 + u;
                if (kk >= KG) break;
                const float b = bq[u];
                if (cok && kk + RING < KG) bq[u] = eb[(int64_t)(kk + RING) * 8 * K];
#pragma unroll
                for (int m = 0; m < MS; ++m) {
                    const float a = Cs[(m * 16 + rl) * CSW + kk * 4 + g];
                    acc[m] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[m], 0, 0, 0);
                }
            }
        }
        if (cok) {
#pragma unroll
            for (int m = 0; m < MS; ++m)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int row = m * 16 + 4 * g + q;
                    const float v = acc[m][q] * rowu[row];
                    if (col < K)
                        Us[row * K + col].x = v;
                    else
                        Us[row * K + col - K].y = v;
                }
        }
    }
}

// The same product with this wave's B fragments already in registers (one U column tile per
// wave: ucol = 16 wave + lane % 16; KG = Wp / 4 k-steps).
template <int BM, int KG>
__device__ __forceinline__ void u_mfma_reg(const float *Cs, int CSW, const float (&ereg)[KG],
                                           int K, const float *rowu, float2 *Us, bool uact,
                                           int ucol) {
    constexpr int MS = BM / 16;
    if (!uact) return;
    const int lane = threadIdx.x & 63, g = lane >> 4, rl = lane & 15;
    f32x4 acc[MS];
#pragma unroll
    for (int m = 0; m < MS; ++m) acc[m] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k0 = 0; k0 < KG; k0 += 4) {
        float a[4][MS];                            // four k-steps of A reads before the MFMAs
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int m = 0; m < MS; ++m)
                a[t][m] = (k0 + t < KG) ? Cs[(m * 16 + rl) * CSW + (k0 + t) * 4 + g] : 0.f;
        asm volatile("" ::: "memory");
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int m = 0; m < MS; ++m)
                if (k0 + t < KG)
                    acc[m] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t][m], ereg[k0 + t], acc[m],
                                                                  0, 0, 0);
    }
    if (ucol < 2 * K) {
#pragma unroll
        for (int m = 0; m < MS; ++m)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = m * 16 + 4 * g + q;
                const float v = acc[m][q] * rowu[row];
                if (ucol < K)
                    Us[row * K + ucol].x = v;
                else
                    Us[row * K + ucol - K].y = v;
            }
    }
}

// Reductions inside each 16-lane DPP row (xor 1, xor 2, half-mirror, mirror): every lane of the
// row ends with the row's result.  Every lane must be active.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    return __builtin_bit_cast(
        float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float row16_max(float v) {
    v = fmaxf(v, dpp_f<0xB1>(v));     // quad_perm [1,0,3,2]
    v = fmaxf(v, dpp_f<0x4E>(v));     // quad_perm [2,3,0,1]
    v = fmaxf(v, dpp_f<0x141>(v));    // row_half_mirror
    return fmaxf(v, dpp_f<0x140>(v)); // row_mirror
}
__device__ __forceinline__ float row16_sum(float v) {
    v += dpp_f<0xB1>(v);
    v += dpp_f<0x4E>(v);
    v += dpp_f<0x141>(v);
    return v + dpp_f<0x140>(v);
}
// Sum over aligned groups of a power-of-two number of consecutive lanes by DPP without branches:
// xor 1 and xor 2 inside quads, then the half-row and row mirrors (each step adds two groups that
// are already uniform); step t counts with weight f[t] = 1 while the group is wider than 2^t
// lanes, else 0 (x * 0 + v = v exactly for finite x), so groups up to 16 lanes end here and wider
// ones continue with xor 16, 32.  Every lane ends with its group's sum; every lane must be active.
__device__ __forceinline__ float lanes_sum_dpp(float v, const float (&f)[4]) {
    v = fmaf(dpp_f<0xB1>(v), f[0], v);
    v = fmaf(dpp_f<0x4E>(v), f[1], v);
    v = fmaf(dpp_f<0x141>(v), f[2], v);
    return fmaf(dpp_f<0x140>(v), f[3], v);
}
// Exchange with lane ^ 16 inside each 32-lane half (ds_swizzle, bit mode: and 0x1f, xor 0x10).
__device__ __forceinline__ float swz_xor16(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_ds_swizzle(__builtin_bit_cast(int, v),
                                                                 0x401F));
}
// Reductions over groups of `width` consecutive lanes: 16-lane rows by DPP, wider groups add
// cross-row shuffles.
template <typename T>
__device__ __forceinline__ T rows_max(T v, int width) {
    if constexpr (sizeof(T) == 4) {
        if (width >= 16) {
            v = row16_max(v);
            if (width >= 32) v = fmaxf(v, swz_xor16(v));
            if (width >= 64) v = fmaxf(v, __shfl_xor(v, 32));
            return v;
        }
    }
    return group_max(v, width);
}
template <typename T>
__device__ __forceinline__ T rows_sum(T v, int width) {
    if constexpr (sizeof(T) == 4) {
        if (width >= 16) {
            v = row16_sum(v);
            if (width >= 32) v += swz_xor16(v);
            if (width >= 64) v += __shfl_xor(v, 32);
            return v;
        }
    }
    return group_sum(v, width);
}
template <typename T>
__device__ __forceinline__ T fast_exp(T x) {
    if constexpr (sizeof(T) == 4) return __expf(x); else return exp(x);
}
template <typename T>
__device__ __forceinline__ T fast_log(T x) {
    if constexpr (sizeof(T) == 4) return __logf(x); else return log(x);
}

// The row-wise part of tile_post: log-sum-exp, posteriors (left in Cs, zero on padding rows and
// columns), the per-row sums and the posterior queries.
template <int P, int BM, int DPT>
__device__ __forceinline__ void tile_rows(const PassArgs &A, int CSW, typename PT<P>::CT *Cs,
                                          const float *lr32, int64_t r0, int rows,
                                          PassAcc<DPT> &acc) {
    typedef typename PT<P>::CT CT;
    constexpr int TPR = kThreads / BM;            // threads per row
    const int tid = threadIdx.x;
    {
        const int r = tid / TPR, sub = tid % TPR;
        const bool valid = r < rows;
        CT *crow = Cs + r * CSW;
        CT lse;
        if (A.flags & PF_LOAD_LSE) {
            lse = valid ? (CT)A.lse[r0 + r] : (CT)0;
        } else {
            CT m = -INFINITY;
            for (int i = sub; i < A.W; i += TPR) m = fmax(m, crow[i]);
            m = rows_max(m, TPR);
            CT s = 0;
            for (int i = sub; i < A.W; i += TPR) s += fast_exp(crow[i] - m);
            s = rows_sum(s, TPR);
            lse = m + fast_log(s);
        }
        CT wc = 0;
        CT b1 = -INFINITY, b2 = -INFINITY;
        int i1 = 0x7fffffff;
        const bool query = (A.flags & PF_QUERY) != 0;
        const int64_t qrow = r0 + r - A.row_begin;
        for (int i = sub; i < A.Wp; i += TPR) {
            const CT l = crow[i];
            CT w = 0;
            if (i < A.W && valid) {
                w = fast_exp(l - lse);
                if (w > (CT)0) {
                    const CT lr = (P == P_F64) ? (CT)A.logrho64[i] : (CT)lr32[i];
                    wc += w * (l - lr);
                }
                if (query) {
                    if (A.post) A.post[qrow * A.W + i] = (float)w;
                    if (l > b1) {
                        b2 = b1;
                        b1 = l;
                        i1 = i;
                    } else if (l > b2) {
                        b2 = l;
                    }
                }
            }
            crow[i] = valid ? w : (CT)0;
        }
        wc = rows_sum(wc, TPR);
        if (query) {
            for (int o = TPR >> 1; o > 0; o >>= 1) {
                const CT ob1 = __shfl_xor(b1, o, TPR), ob2 = __shfl_xor(b2, o, TPR);
                const int oi1 = __shfl_xor(i1, o, TPR);
                if (ob1 > b1 || (ob1 == b1 && oi1 < i1)) {
                    b2 = fmax(b1, ob2);
                    b1 = ob1;
                    i1 = oi1;
                } else {
                    b2 = fmax(b2, ob1);
                }
            }
            if (sub == 0 && valid) {
                if (A.argmax) A.argmax[qrow] = i1;
                if (A.margin) {
                    const CT w1 = fast_exp(b1 - lse), w2 = (A.W > 1) ? fast_exp(b2 - lse) : (CT)0;
                    A.margin[qrow] = (float)(w1 - w2);
                }
            }
        }
        if (sub == 0 && valid) {
            acc.lse += (double)lse;
            acc.wc += (double)wc;                     // sum_i w_ji (l_ji - log rho_i)
            acc.rows += 1.0;
            if (A.flags & PF_STORE_LSE) A.lse[r0 + r] = (double)lse;
        }
    }
}

// tile_rows for windows of at most 64 offsets and no posterior queries: 16 threads per row (the
// first 16 BM threads), each with 4 consecutive log-weights in registers (one 16-byte LDS read
// and write), one exponential per entry (w = exp(l - m) / s with s = sum exp(l - m)) and DPP
// row reductions.  Columns W .. 63 get zero posteriors.
template <int BM, int DPT>
__device__ __forceinline__ void tile_rows_short(const PassArgs &A, int CSW, float *Cs,
                                                const float *lr32, int64_t r0, int rows,
                                                PassAcc<DPT> &acc, uint8_t *wb = nullptr,
                                                const float4 *lrv = nullptr) {
    static_assert(16 * BM <= kThreads, "16 threads per row");
    const int tid = threadIdx.x;
    if (tid >= 16 * BM) return;                    // (whole waves)
    const int r = tid >> 4, i0 = 4 * (tid & 15);
    const bool valid = r < rows;
    float4 *cp = (float4 *)(Cs + r * CSW + i0);
    const float4 l4 = *cp;
    const float l[4] = {l4.x, l4.y, l4.z, l4.w};
    float m = -INFINITY;
#pragma unroll
    for (int t = 0; t < 4; ++t)
        if (i0 + t < A.W) m = fmaxf(m, l[t]);
    m = row16_max(m);
    float e[4], s = 0.f;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        e[t] = i0 + t < A.W ? __expf(l[t] - m) : 0.f;
        s += e[t];
    }
    s = row16_sum(s);
    const float lse = m + __logf(s), inv = 1.0f / s;
    const float4 lr4 = lrv ? *lrv : *(const float4 *)(lr32 + i0);
    const float lr[4] = {lr4.x, lr4.y, lr4.z, lr4.w};
    float w[4], wc = 0.f;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        w[t] = valid ? e[t] * inv : 0.f;
        if (w[t] > 0.f) wc += w[t] * (l[t] - lr[t]);
    }
    *cp = make_float4(w[0], w[1], w[2], w[3]);
    if (wb) {                                      // bf16 hi + lo planes of the row (256 B)
        bf16x4 h, lo;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            h[t] = (__bf16)w[t];
            lo[t] = (__bf16)(w[t] - (float)h[t]);
        }
        *(bf16x4 *)(wb + r * 256 + 2 * i0) = h;
        *(bf16x4 *)(wb + r * 256 + 128 + 2 * i0) = lo;
    }
    wc = row16_sum(wc);
    if ((tid & 15) == 0 && valid) {
        acc.lse += (double)lse;
        acc.wc += (double)wc;                     // sum_i w_ji (l_ji - log rho_i)
        acc.rows += 1.0;
        if (A.flags & PF_STORE_LSE) A.lse[r0 + r] = (double)lse;
    }
}

// W_t column sums of the posteriors of one tile (after tile_rows and a barrier).
template <int P, int DPT>
__device__ __forceinline__ void tile_wsum(const PassArgs &A, int CSW,
                                          const typename PT<P>::CT *Cs, int rows,
                                          PassAcc<DPT> &acc) {
    typedef typename PT<P>::CT CT;
    const int tid = threadIdx.x;
    for (int c = 0; c < 2; ++c) {
        const int i = tid + c * kThreads;
        if (i < A.Wp) {
            CT s = 0;
            int j = 0;
            for (; j + 8 <= rows; j += 8) {
                CT v[8];
#pragma unroll
                for (int t = 0; t < 8; ++t) v[t] = Cs[(j + t) * CSW + i];
#pragma unroll
                for (int t = 0; t < 8; ++t) s += v[t];
            }
            for (; j < rows; ++j) s += Cs[j * CSW + i];
            acc.W[c] += (double)s;
        }
    }
}

// a4 + a5 for one tile whose log-weights l' = coef C + log rho are in Cs (BM x CSW) and whose
// observation rows are in Vs: per-row log-sum-exp and posteriors, then (with PF_ACC_M) the W_t
// column sums, U = w E and the M-step accumulation S_d += sum_j U_{j,kbar_d} v_jd.
// KG > 0: the U B-fragments of this wave are in registers (ereg); KG == 0: they stream from L2.
template <int P, int BM, int DPT, int KG>
__device__ __forceinline__ void tile_post(const PassArgs &A, const PassLds &LY, const uint8_t *Vs,
                                          typename PT<P>::CT *Cs, typename PT<P>::CT2 *Us,
                                          const float *rowu, const float *lr32, int64_t r0,
                                          int rows, PassAcc<DPT> &acc,
                                          const float (&ereg)[KG > 0 ? KG : 1], bool uact,
                                          int ucol) {
    typedef typename PT<P>::CT CT;
    typedef typename PT<P>::CT2 CT2;
    const int tid = threadIdx.x;
    tile_rows<P, BM, DPT>(A, LY.CSW, Cs, lr32, r0, rows, acc);
    if (!(A.flags & PF_ACC_M)) return;
    lds_barrier();
    tile_wsum<P, DPT>(A, LY.CSW, Cs, rows, acc);
    // U_jk = sum_i w_ji exp(+i k theta_i), scaled back to the rows' storage scale
    if constexpr (P == P_F64) {
        for (int p = tid; p < rows * A.K; p += kThreads) {
            const int j = p / A.K, k = p - j * A.K;
            const double *wr = Cs + j * LY.CSW;
            double ur = 0, ui = 0;
            for (int i = 0; i < A.W; ++i) {
                const double2 e = A.E64[i * A.K + k];
                ur = fma(wr[i], e.x, ur);
                ui = fma(wr[i], e.y, ui);
            }
            Us[p] = make_double2(ur, ui);
        }
    } else if constexpr (KG > 0) {
        u_mfma_reg<BM, KG>(Cs, LY.CSW, ereg, A.K, rowu, Us, uact, ucol);
    } else {
        u_mfma<BM>(Cs, LY.CSW, A.E2, A.Wp, A.K, rowu, Us);
    }
    lds_barrier();
    // M-step: S_d += sum_j U_{j, kbar_d} v_jd (complex product, no conjugate)
#pragma unroll
    for (int c = 0; c < DPT; ++c) {
        const int d = tid + c * kThreads;
        if (d < A.D) {
            const int k = d / A.Q;
            CT sr = 0, si = 0;
            for (int j = 0; j < rows; ++j) {
                CT2 v;
                if constexpr (P == P_F64) {
                    v = load_v<P>(Vs + j * LY.RS, d, A.Dp);
                } else {
                    v = load_v32<P>(Vs + j * LY.RS, d, A.Dp);
                }
                const CT2 u = Us[j * A.K + k];
                sr += u.x * v.x - u.y * v.y;
                si += u.x * v.y + u.y * v.x;
            }
            acc.S[c].x += (double)sr;
            acc.S[c].y += (double)si;
        }
    }
}

// Per-workgroup partials: S (2D), W (Wp), sum lse', sum w*C, rows, 0.
// The per-workgroup scalars of a pass (sum of per-row log-sum-exps, sum of w C, rows) summed in a
// fixed order (a 64-lane butterfly, which leaves every lane with the same sum, then the waves in
// order) and stored at out[0 .. 3] (the w C sum divided by coef, then a zero).  sh: 3 doubles per
// wave of LDS that no wave still uses.
__device__ __forceinline__ void put_pass_scalars(double *out, double lse, double wc, double rows,
                                                 double coef, double *sh) {
    double v[3] = {lse, wc, rows};
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) v[q] += __shfl_xor(v[q], o);
    const int t = threadIdx.x;
    if ((t & 63) == 0)
#pragma unroll
        for (int q = 0; q < 3; ++q) sh[(t >> 6) * 3 + q] = v[q];
    __syncthreads();
    if (t == 0) {
        double r[3] = {sh[0], sh[1], sh[2]};
        for (int w = 1; w < kThreads / 64; ++w)
#pragma unroll
            for (int q = 0; q < 3; ++q) r[q] += sh[w * 3 + q];
        out[0] = r[0];
        out[1] = r[1] / coef;
        out[2] = r[2];
        out[3] = 0.0;
    }
}

template <int DPT>
__device__ __forceinline__ void write_partials(const PassArgs &A, PassAcc<DPT> &acc,
                                               uint8_t *smem) {
    const int tid = threadIdx.x;
    double *Pp = A.partials + (int64_t)blockIdx.x * A.ncols;
    if (A.flags & PF_ACC_M) {
#pragma unroll
        for (int c = 0; c < DPT; ++c) {
            const int d = tid + c * kThreads;
            if (d < A.D) {
                Pp[2 * d] = acc.S[c].x;
                Pp[2 * d + 1] = acc.S[c].y;
            }
        }
        for (int c = 0; c < 2; ++c) {
            const int i = tid + c * kThreads;
            if (i < A.Wp) Pp[2 * A.D + i] = acc.W[c];
        }
    } else {
        for (int i = tid; i < 2 * A.D + A.Wp; i += kThreads) Pp[i] = 0.0;
    }
    __syncthreads();
    // (sum_j lse'_j, sum_j sum_i w_ji C_ji, rows)
    put_pass_scalars(Pp + 2 * A.D + A.Wp, acc.lse, acc.wc, acc.rows, A.coef, (double *)smem);
}

// Global-to-LDS copy of BYTES (16 or 4) per lane: lane l's bytes land at lds_dst + BYTES l (lds_dst
// wave-uniform).  Written as inline assembly so that the compiler does not make every later LDS
// access wait for it (it cannot tell which LDS bytes such a copy writes, so with the builtin it
// waits for all vector-memory operations before reading any LDS); its completion is tracked with
// explicit vector-memory counts and a barrier before the bytes are read.  M0 is restored.
template <int BYTES>
__device__ __forceinline__ void dma_to_lds(const void *src, void *lds_dst) {
    static_assert(BYTES == 16 || BYTES == 4, "dword or dwordx4 copies");
    // (uniform by construction; read from the first lane so that it sits in a scalar register)
    const uint32_t m = __builtin_amdgcn_readfirstlane(
        (uint32_t)(uintptr_t)(__attribute__((address_space(3))) void *)lds_dst);
    uint32_t save;
    if constexpr (BYTES == 16)
        asm volatile("s_mov_b32 %0, m0\n\ts_mov_b32 m0, %2\n\ts_nop 0\n\t"
                     "global_load_lds_dwordx4 %1, off\n\ts_mov_b32 m0, %0"
                     : "=&s"(save) : "v"(src), "s"(m) : "memory");
    else
        asm volatile("s_mov_b32 %0, m0\n\ts_mov_b32 m0, %2\n\ts_nop 0\n\t"
                     "global_load_lds_dword %1, off\n\ts_mov_b32 m0, %0"
                     : "=&s"(save) : "v"(src), "s"(m) : "memory");
}

// Asynchronous copy of one row tile into an LDS tile buffer with the direct global-to-LDS load
// (16 bytes per lane; a wave's 64 lanes fill 1 KB of LDS in lane order).  Rows are whole 1 KB
// chunks (rowbytes is a multiple of 1024 here); wave w copies chunks w, w + 8, ...  Completion
// is awaited with s_waitcnt before the barrier that precedes the first read of the buffer.
__device__ __forceinline__ void dma_issue_tile(const PassArgs &A, int64_t tile, int BM,
                                              uint8_t *buf, int RS) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t r0 = A.row_begin + tile * BM;
    const int rows = (int)((A.row_end - r0) < BM ? (A.row_end - r0) : BM);
    const int cpr = (int)(A.rowbytes >> 10);
    const int nch = rows * cpr;
    for (int c = wave; c < nch; c += kThreads / 64) {
        const int r = c / cpr, k = c - r * cpr;
        dma_to_lds<16>(A.V + (r0 + r) * A.rowbytes + k * 1024 + lane * 16, buf + r * RS + k * 1024);
    }
}

// General E(+M) pass: the template is streamed from L2 in B-fragment order; the 8 waves split the
// window's 16-column tiles (WN of them) and the tile's 16-row blocks (WM of them).  LD = 1: the
// row tile is double-buffered in LDS by direct global-to-LDS copies (rows of whole KiB); LD = 0:
// it is staged through registers.
template <int P, int BM, int WM, int LD>
__global__ __launch_bounds__(kThreads) void pass_kernel(PassArgs A) {
    typedef typename PT<P>::CT CT;
    typedef typename PT<P>::CT2 CT2;
    constexpr int MS = BM / 16;
    constexpr int MSW = (MS / WM) > 0 ? MS / WM : 1;
    // column tiles per GEMM pass and template prefetch depth (k-steps); the register-staged
    // variants keep 64 VGPRs of tile prefetch and so use the lighter setting
    constexpr int NTW = (WM == 1 && LD) ? ((MSW >= 2 || P != P_F32) ? 2 : 3) : 1;
    constexpr int PD = (LD && P == P_F32) ? 4 : 2;

    if ((A.flags & PF_CHECK_STOP) && *A.stopped) return;

    extern __shared__ __align__(16) uint8_t smem[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const PassLds LY = pass_lds(P, BM, A.K, A.Dp, A.Wp, LD ? 2 : 1);
    CT *Cs = (CT *)(smem + LY.off_c);
    CT2 *Us = (CT2 *)(smem + LY.off_u);
    CT *rowf = (CT *)(smem + LY.off_f);
    float *rowu = (float *)(smem + LY.off_f + BM * sizeof(CT));
    float *lrs = (float *)(smem + LY.off_lr);
    for (int i = tid; i < A.Wp; i += kThreads) lrs[i] = A.logrho32[i];

    const int64_t ntiles = (A.row_end - A.row_begin + BM - 1) / BM;
    const int NT = A.Wp / 16;
    const int WN = 8 / WM;
    const int wn = wave % WN, wm = wave / WN;

    PassAcc<kMaxDPerThread> acc;
    acc.init();
    const float tsc = (P == P_F64 || P == P_F32) ? 1.0f : *A.tscale;
    TileLoader<LD ? 1 : kRegTileChunks> ld;

    int64_t tile = blockIdx.x;
    int buf = 0;
    if (tile < ntiles) {
        if constexpr (LD) dma_issue_tile(A, tile, BM, smem, LY.RS);
        else ld.issue(A, tile, BM);
    }
    for (; tile < ntiles; tile += gridDim.x, buf ^= 1) {
        const int64_t r0 = A.row_begin + tile * BM;
        const int rows = (int)((A.row_end - r0) < BM ? (A.row_end - r0) : BM);
        uint8_t *Vs = smem + ((LD && buf) ? LY.off_v1 : 0);
        if constexpr (LD) {
            __builtin_amdgcn_s_waitcnt(0);                  // this tile's copy has landed
            __syncthreads();
            if (tile + gridDim.x < ntiles)
                dma_issue_tile(A, tile + gridDim.x, BM, smem + (buf ? 0 : LY.off_v1), LY.RS);
        } else {
            lds_barrier();                                // previous tile fully consumed
            ld.store(Vs, LY.RS, BM, A.rowbytes);
        }
        for (int j = tid; j < BM; j += kThreads) {
            CT f = (CT)A.coef;
            float u = 1.0f;
            if (P != P_F64 && A.rowscale && j < rows) {
                u = A.rowscale[r0 + j];
                f *= (CT)u * (CT)tsc;
            }
            rowf[j] = f;
            rowu[j] = u;
        }
        lds_barrier();
        if constexpr (!LD)
            if (tile + gridDim.x < ntiles) ld.issue(A, tile + gridDim.x, BM);

        // ---- a3: correlations C and log-weights l' = coef * C + log rho  -> Cs
        if constexpr (P == P_F64) {
            const double *Td = (const double *)A.Thi;
            const int nq = BM * A.Wp / kThreads;
            if (LD && kThreads % A.Wp == 0 && nq * kThreads == BM * A.Wp && nq <= 4) {
                // every output of a thread lies in one window column (col = tid % Wp, rows
                // tid / Wp + q kThreads / Wp): one read of the template column serves all of
                // them; eight reals read at a time (the LDS-staged form only: the register-staged
                // one has no registers to spare)
                const int col = tid % A.Wp, r0 = tid / A.Wp, rstep = kThreads / A.Wp;
                const double *tc = Td + col;
                double sq[4] = {0.0, 0.0, 0.0, 0.0};
                int k = 0;
                for (; k + 8 <= A.Dp; k += 8) {
                    double t[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) t[u] = tc[(int64_t)(k + u) * A.Wp];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        if (q >= nq) break;
                        const double *vr = (const double *)(Vs + (r0 + q * rstep) * LY.RS);
#pragma unroll
                        for (int u = 0; u < 8; ++u) sq[q] = fma(vr[k + u], t[u], sq[q]);
                    }
                }
                for (; k < A.Dp; ++k) {
                    const double t = tc[(int64_t)k * A.Wp];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        if (q >= nq) break;
                        const double *vr = (const double *)(Vs + (r0 + q * rstep) * LY.RS);
                        sq[q] = fma(vr[k], t, sq[q]);
                    }
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (q >= nq) break;
                    Cs[(r0 + q * rstep) * LY.CSW + col] = sq[q] * A.coef + A.logrho64[col];
                }
            } else
            // (the template column is read from global memory 16 reals at a time, all 16 reads
            // issued before the products, which run in four chains added at the end)
            for (int o = tid; o < BM * A.Wp; o += kThreads) {
                const int r = o / A.Wp, col = o - r * A.Wp;
                const double *vr = (const double *)(Vs + r * LY.RS);
                const double *tc = Td + col;
                double s4[4] = {0.0, 0.0, 0.0, 0.0};
                int k = 0;
                for (; k + 16 <= A.Dp; k += 16) {
                    double t[16];
#pragma unroll
                    for (int u = 0; u < 16; ++u) t[u] = tc[(int64_t)(k + u) * A.Wp];
#pragma unroll
                    for (int u = 0; u < 16; ++u) s4[u & 3] = fma(vr[k + u], t[u], s4[u & 3]);
                }
                for (; k < A.Dp; ++k) s4[0] = fma(vr[k], tc[(int64_t)k * A.Wp], s4[0]);
                const double s = (s4[0] + s4[1]) + (s4[2] + s4[3]);
                Cs[r * LY.CSW + col] = s * A.coef + A.logrho64[col];
            }
        } else {
            if (wm < WM) {
                for (int nt0 = wn; nt0 < NT; nt0 += WN * NTW) {
                    f32x4 c4[NTW][MSW];
                    gemm_ntiles<P, MSW, WM, NTW, PD>(c4, Vs, LY.RS, wm, lane, nt0, WN, NT, A.Dp,
                                                     A.Thi, A.Tlo);
#pragma unroll
                    for (int n = 0; n < NTW; ++n) {
                        const int nt = nt0 + n * WN;
                        if (nt >= NT) continue;
                        const int col = nt * 16 + (lane & 15);
                        const float lr = lrs[col];
#pragma unroll
                        for (int m = 0; m < MSW; ++m) {
                            const int rb = (wm + m * WM) * 16 + 4 * (lane >> 4);
#pragma unroll
                            for (int q = 0; q < 4; ++q)
                                Cs[(rb + q) * LY.CSW + col] = c4[n][m][q] * rowf[rb + q] + lr;
                        }
                    }
                }
            }
        }
        lds_barrier();
        const float nore[1] = {0.f};
        tile_post<P, BM, kMaxDPerThread, 0>(A, LY, Vs, Cs, Us, rowu, lrs, r0, rows, acc, nore,
                                            false, 0);
    }
    if (A.partials) write_partials(A, acc, smem);
}

// ------------------------------------------------------------------------------------------
// K-split E(+M) pass for windows whose whole template fits in the register file: wave w holds
// the template rows of its K-slice (KSS k-steps of 32 reals) for all NT column tiles, loaded once
// per launch; per tile every wave contracts its K-slice of the tile's rows against it, and the
// eight partial correlations are summed in a fixed order through LDS (waves 4-7 into 0-3, then
// ((s0 + s1) + s2) + s3), so the result does not depend on scheduling.

// The inputs a template-in-registers pass builds its template from, staged in LDS once per
// workgroup (every workgroup reads the same few KiB; read straight from global memory inside the
// template loops, those reads queue on the same cache lines and take tens of microseconds): a_t
// as FP32 (Re, Im) pairs (D <= 4 kThreads entries) at st, then the window's phase rows E2 (Wp
// rows of [cos | sin] x K floats, Wp 2K <= 16 kThreads).  Returns max |Re a_d|, |Im a_d| to every
// thread (sh8: 8 doubles of LDS); its barrier publishes the staged tables.
constexpr int kStageA = 4, kStageE = 16;
__device__ double stage_a_e2(const PassArgs &A, uint8_t *st, double *sh8) {
    float2 *as = (float2 *)st;
    float *es = (float *)(st + 8 * A.D);
    const int t = threadIdx.x, ne = A.Wp * 2 * A.K;
    double ar[kStageA], ai[kStageA];
    float ev[kStageE];
#pragma unroll
    for (int c = 0; c < kStageA; ++c) {
        const int d = t + c * kThreads;
        ar[c] = d < A.D ? A.a[2 * d] : 0.0;
        ai[c] = d < A.D ? A.a[2 * d + 1] : 0.0;
    }
#pragma unroll
    for (int c = 0; c < kStageE; ++c) {
        const int x = t + c * kThreads;
        ev[c] = x < ne ? A.E2[x] : 0.f;
    }
    double amax = 0.0;
#pragma unroll
    for (int c = 0; c < kStageA; ++c) {
        const int d = t + c * kThreads;
        amax = fmax(amax, fmax(fabs(ar[c]), fabs(ai[c])));
        if (d < A.D) as[d] = make_float2((float)ar[c], (float)ai[c]);
    }
#pragma unroll
    for (int c = 0; c < kStageE; ++c) {
        const int x = t + c * kThreads;
        if (x < ne) es[x] = ev[c];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) amax = fmax(amax, __shfl_xor(amax, o));
    if ((t & 63) == 0) sh8[t >> 6] = amax;
    __syncthreads();
    double r = sh8[0];
#pragma unroll
    for (int w = 1; w < kThreads / 64; ++w) r = fmax(r, sh8[w]);
    return r;
}
__host__ __device__ inline int stage_a_e2_bytes(int D, int Wp, int K) { return 8 * D + 8 * Wp * K; }

// One B fragment of the rotated template from the staged tables: entries d0 .. d0 + 3 at window
// column i (phase row Ei), T = (Re, Im)(a_d conj(exp(+i k_d theta_i))) sc with k_d = d / Q
// (rq = 1 / Q; (d + 1/2) / Q sits at least 1 / (2 Q) from an integer, far beyond the rounding of
// the product), split into 16-bit hi + lo; entries at or past D are zero.  Branch-free: the reads
// are clamped into the tables and the entries selected afterwards, so that the reads of a whole
// template slice can be in flight together.
template <typename H>
__device__ __forceinline__ void tpl_frag(const float2 *as, const float *Ei, int d0, int D, int K,
                                         float rq, float sc, u32x4 &hi, u32x4 &lo) {
    H hv[8], lv[8];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int d = d0 + e;
        const bool ok = d < D;
        const int dc = ok ? d : D - 1;
        const int k = (int)(((float)dc + 0.5f) * rq);
        const float2 a = as[dc];
        const float er = Ei[k], ei = Ei[K + k];
        const float tre = ok ? (a.x * er + a.y * ei) * sc : 0.f;
        const float tim = ok ? (a.y * er - a.x * ei) * sc : 0.f;
        hv[2 * e] = (H)tre;
        hv[2 * e + 1] = (H)tim;
        lv[2 * e] = (H)(tre - (float)hv[2 * e]);
        lv[2 * e + 1] = (H)(tim - (float)hv[2 * e + 1]);
    }
    hi = __builtin_bit_cast(u32x4, hv);
    lo = __builtin_bit_cast(u32x4, lv);
}

// The same fragment when the four entries share one frequency (Q % 4 == 0): ar, ai are
// Re, Im a_d of the four entries already multiplied by sc (a power of two, so every product is
// what scaling it afterwards gives), er, ei the phase at their frequency.
template <typename H>
__device__ __forceinline__ void tpl_frag4(const float ar[4], const float ai[4], float er, float ei,
                                          u32x4 &hi, u32x4 &lo) {
    H hv[8], lv[8];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const float tre = ar[e] * er + ai[e] * ei;
        const float tim = ai[e] * er - ar[e] * ei;
        hv[2 * e] = (H)tre;
        hv[2 * e + 1] = (H)tim;
        lv[2 * e] = (H)(tre - (float)hv[2 * e]);
        lv[2 * e + 1] = (H)(tim - (float)hv[2 * e + 1]);
    }
    hi = __builtin_bit_cast(u32x4, hv);
    lo = __builtin_bit_cast(u32x4, lv);
}

struct KsLds {
    int RS, CSW;
    int off_v1, off_red, off_c, off_u, off_f, off_lr, total;
};
__host__ __device__ inline KsLds ks_lds(int prec, int BM, int NT, int K, int Dp, int Wp) {
    KsLds l;
    l.RS = (int)row_bytes(prec, Dp) + 16;
    l.CSW = Wp + 4;                                         // conflict-free U operand reads
    l.off_v1 = align_up(BM * l.RS, 16);                     // second tile buffer
    l.off_red = align_up(2 * BM * l.RS, 16);
    l.off_c = align_up(l.off_red + 4 * (BM / 16) * NT * 64 * 16, 16);
    l.off_u = align_up(l.off_c + BM * l.CSW * 4, 16);
    l.off_f = align_up(l.off_u + BM * K * 8, 16);
    l.off_lr = align_up(l.off_f + 2 * BM * 4, 16);
    l.total = l.off_lr + Wp * 4 + 16;
    return l;
}

template <int P>
__host__ __device__ constexpr int bytes_per_real() {
    return P == P_BF16X3 ? 4 : (P == P_F32 ? 4 : 2);
}

// Wave-wide reductions: the 16-lane row reductions (row16_*), then the four row results
// combined in a fixed order through readlane.  Every lane must be active.
__device__ __forceinline__ float rl_f(float v, int lane) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}
__device__ __forceinline__ float wave_max_f(float v) {
    v = fmaxf(v, dpp_f<0xB1>(v));     // quad_perm [1,0,3,2]
    v = fmaxf(v, dpp_f<0x4E>(v));     // quad_perm [2,3,0,1]
    v = fmaxf(v, dpp_f<0x141>(v));    // row_half_mirror
    v = fmaxf(v, dpp_f<0x140>(v));    // row_mirror
    return fmaxf(fmaxf(rl_f(v, 0), rl_f(v, 16)), fmaxf(rl_f(v, 32), rl_f(v, 48)));
}
// H independent wave reductions, their steps interleaved.
template <int H>
__device__ __forceinline__ void wave_max_fn(float (&v)[H]) {
#pragma unroll
    for (int h = 0; h < H; ++h) v[h] = fmaxf(v[h], dpp_f<0xB1>(v[h]));
#pragma unroll
    for (int h = 0; h < H; ++h) v[h] = fmaxf(v[h], dpp_f<0x4E>(v[h]));
#pragma unroll
    for (int h = 0; h < H; ++h) v[h] = fmaxf(v[h], dpp_f<0x141>(v[h]));
#pragma unroll
    for (int h = 0; h < H; ++h) v[h] = fmaxf(v[h], dpp_f<0x140>(v[h]));
#pragma unroll
    for (int h = 0; h < H; ++h)
        v[h] = fmaxf(fmaxf(rl_f(v[h], 0), rl_f(v[h], 16)), fmaxf(rl_f(v[h], 32), rl_f(v[h], 48)));
}
template <int H>
__device__ __forceinline__ void wave_sum_fn(float (&v)[H]) {
#pragma unroll
    for (int h = 0; h < H; ++h) v[h] += dpp_f<0xB1>(v[h]);
#pragma unroll
    for (int h = 0; h < H; ++h) v[h] += dpp_f<0x4E>(v[h]);
#pragma unroll
    for (int h = 0; h < H; ++h) v[h] += dpp_f<0x141>(v[h]);
#pragma unroll
    for (int h = 0; h < H; ++h) v[h] += dpp_f<0x140>(v[h]);
#pragma unroll
    for (int h = 0; h < H; ++h)
        v[h] = (rl_f(v[h], 0) + rl_f(v[h], 16)) + (rl_f(v[h], 32) + rl_f(v[h], 48));
}
__device__ __forceinline__ float wave_sum_f(float v) {
    v += dpp_f<0xB1>(v);
    v += dpp_f<0x4E>(v);
    v += dpp_f<0x141>(v);
    v += dpp_f<0x140>(v);
    return (rl_f(v, 0) + rl_f(v, 16)) + (rl_f(v, 32) + rl_f(v, 48));
}

// a4 + a5 of the K-split pass without posterior queries: wave w owns the rows w, w + 8, ... of
// the tile with one window column per lane (Wp <= 64).  It sums the eight K-slices of its rows,
// forms the log-weights, their log-sum-exp and the posteriors in registers, adds the posteriors
// to its per-lane W_t accumulator and leaves them in Cs; then U = w E on matrix cores and the
// M-step over the tile's rows.
template <int P, int BM, int NT, int DPT, int KG>
__device__ __forceinline__ void ks_post(const PassArgs &A, const KsLds &LY, const uint8_t *Vs,
                                        const f32x4 *red, float *Cs, float2 *Us,
                                        const float *rowf, const float *rowu, const float *lrs,
                                        int64_t r0, int rows, PassAcc<DPT> &acc, double &accWl,
                                        const float (&ereg)[KG], bool uact, int ucol) {
    constexpr int MS = BM / 16;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int col = lane, nt = lane >> 4;
    const bool cval = col < A.W;
    const float lr = col < A.Wp ? lrs[col] : -INFINITY;
    // this wave's H = BM / 8 rows (wave, wave + 8, ...), their reductions interleaved step by step
    constexpr int H = BM / 8;
    float l[H], lse[H], w[H], wc[H];
    bool rv[H];
#pragma unroll
    for (int h = 0; h < H; ++h) {
        const int r = wave + 8 * h;
        rv[h] = r < rows;
        const int m = r >> 4, rr = r & 15;
        const int ln = (rr >> 2) * 16 + (col & 15), q = rr & 3;
        l[h] = -INFINITY;
        if (cval && rv[h]) {
            float v = red[((0 * MS + m) * NT + nt) * 64 + ln][q];
            v += red[((1 * MS + m) * NT + nt) * 64 + ln][q];
            v += red[((2 * MS + m) * NT + nt) * 64 + ln][q];
            v += red[((3 * MS + m) * NT + nt) * 64 + ln][q];
            l[h] = v * rowf[r] + lr;
        }
    }
    if (A.flags & PF_LOAD_LSE) {
#pragma unroll
        for (int h = 0; h < H; ++h) lse[h] = rv[h] ? (float)A.lse[r0 + wave + 8 * h] : 0.f;
    } else {
        float mx[H], sx[H];
#pragma unroll
        for (int h = 0; h < H; ++h) mx[h] = l[h];
        wave_max_fn<H>(mx);
#pragma unroll
        for (int h = 0; h < H; ++h) sx[h] = (cval && rv[h]) ? __expf(l[h] - mx[h]) : 0.f;
        wave_sum_fn<H>(sx);
#pragma unroll
        for (int h = 0; h < H; ++h) lse[h] = mx[h] + __logf(sx[h]);
    }
#pragma unroll
    for (int h = 0; h < H; ++h) {
        w[h] = (cval && rv[h]) ? __expf(l[h] - lse[h]) : 0.f;
        wc[h] = w[h] > 0.f ? w[h] * (l[h] - lr) : 0.f;
    }
    wave_sum_fn<H>(wc);
    float wsum = 0.f;
#pragma unroll
    for (int h = 0; h < H; ++h) {
        const int r = wave + 8 * h;
        if (col < A.Wp) Cs[r * LY.CSW + col] = w[h];
        wsum += w[h];
        if (lane == 0 && rv[h]) {
            acc.lse += (double)lse[h];
            acc.wc += (double)wc[h];
            acc.rows += 1.0;
            if (A.flags & PF_STORE_LSE) A.lse[r0 + r] = (double)lse[h];
        }
    }
    accWl += (double)wsum;
    if (!(A.flags & PF_ACC_M)) return;
    lds_barrier();
    u_mfma_reg<BM, KG>(Cs, LY.CSW, ereg, A.K, rowu, Us, uact, ucol);
    lds_barrier();
    // M-step: S_d += sum_j U_{j, kbar_d} v_jd, all BM rows unconditionally (rows past the
    // tile's end are masked by a select, so stale LDS contents cannot leak in)
#pragma unroll
    for (int c = 0; c < DPT; ++c) {
        const int d = tid + c * kThreads;
        if (d < A.D) {
            const int k = d / A.Q;
            float sr = 0.f, si = 0.f;
#pragma unroll
            for (int j0 = 0; j0 < BM; j0 += 4) {
                float2 v[4], u[4];                 // four rows of loads before any arithmetic
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    v[t] = load_v32<P>(Vs + (j0 + t) * LY.RS, d, A.Dp);
                    u[t] = Us[(j0 + t) * A.K + k];
                }
                asm volatile("" ::: "memory");
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const bool ok = j0 + t < rows;
                    sr += ok ? u[t].x * v[t].x - u[t].y * v[t].y : 0.f;
                    si += ok ? u[t].x * v[t].y + u[t].y * v[t].x : 0.f;
                }
            }
            acc.S[c].x += (double)sr;
            acc.S[c].y += (double)si;
        }
    }
}

template <int P, int BM, int NT, int KSS, int QRY>
__global__ __launch_bounds__(kThreads) void pass_ks_kernel(PassArgs A) {
    constexpr int MS = BM / 16;
    constexpr int DPT = (KSS * 128 + kThreads - 1) / kThreads;
    constexpr int KG = NT * 4;                              // k-steps of the U product (Wp / 4)
    static_assert(P == P_BF16X3 || P == P_F16 || P == P_BF16, "16-bit MFMA paths only");
    typedef typename std::conditional<P == P_F16, _Float16, __bf16>::type H;

    if ((A.flags & PF_CHECK_STOP) && *A.stopped) return;

    extern __shared__ __align__(16) uint8_t smem[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, rl = lane & 15;
    const KsLds LY = ks_lds(P, BM, NT, A.K, A.Dp, A.Wp);
    f32x4 *red = (f32x4 *)(smem + LY.off_red);
    float *Cs = (float *)(smem + LY.off_c);
    float2 *Us = (float2 *)(smem + LY.off_u);
    float *rowf = (float *)(smem + LY.off_f);
    float *rowu = rowf + BM;
    float *lrs = (float *)(smem + LY.off_lr);
    PassLds PL;                                             // the view tile_post expects
    PL.RS = LY.RS;
    PL.CSW = LY.CSW;
    const int D = A.D, K = A.K;

    // log rho into LDS; template scale from max |Re a|, |Im a| (a power of two, see the
    // storage-scaling note above)
    for (int i = tid; i < A.Wp; i += kThreads) lrs[i] = A.logrho32[i];
    // a_t and the phase rows staged in LDS (the tile buffers' area, first copied into after the
    // barrier that ends the template build)
    const double amax = stage_a_e2(A, smem, (double *)rowf);
    const float2 *as = (const float2 *)smem;
    const float *es = (const float *)(smem + 8 * D);
    const float rq = 1.0f / (float)A.Q;
    float sc = 1.0f, tsc = 1.0f;
    if (amax > 0.0) {
        const int e = ilogb(amax);
        sc = ldexpf(1.0f, scale_target(P) - e);
        tsc = ldexpf(1.0f, e - scale_target(P));
    }

    // this wave's template K-slice for all column tiles, built from a_t in registers:
    // T[r][i] = (Re, Im)(a_d conj(exp(+i k_d theta_i))) * sc, d = r / 2, split into hi + lo
    u32x4 treg[KSS][NT][2];
#pragma unroll
    for (int ks = 0; ks < KSS; ++ks) {
        const int d0 = ((wave * KSS + ks) * 32 + 8 * g) >> 1;        // a multiple of 4
        if (A.Q % 4 == 0 && D % 4 == 0) {           // the four entries share k and validity
            const bool ok = d0 < D;
            const int k = ok ? (int)(((float)d0 + 0.5f) * rq) : 0;
            const float4 a01 = *(const float4 *)(as + (ok ? d0 : 0));
            const float4 a23 = *(const float4 *)(as + (ok ? d0 + 2 : 0));
            const float f = ok ? sc : 0.f;
            const float ar[4] = {a01.x * f, a01.z * f, a23.x * f, a23.z * f};
            const float ai[4] = {a01.y * f, a01.w * f, a23.y * f, a23.w * f};
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const float *Ei = es + (nt * 16 + rl) * 2 * K;
                tpl_frag4<H>(ar, ai, Ei[k], Ei[K + k], treg[ks][nt][0], treg[ks][nt][1]);
            }
        } else {
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                tpl_frag<H>(as, es + (nt * 16 + rl) * 2 * K, d0, D, K, rq, sc, treg[ks][nt][0],
                            treg[ks][nt][1]);
        }
    }
    // B fragments of U = w [Re E | Im E] for this wave's 16-column tile of U
    const int ucol = wave * 16 + rl;
    const bool uact = wave * 16 < 2 * K, uok = ucol < 2 * K;
    float ereg[KG];
#pragma unroll
    for (int kk = 0; kk < KG; ++kk)
        ereg[kk] = uok ? es[uok ? (kk * 4 + g) * 2 * K + ucol : 0] : 0.f;
    __syncthreads();                                        // the staged tables are consumed

    const int64_t ntiles = (A.row_end - A.row_begin + BM - 1) / BM;
    PassAcc<DPT> acc;
    acc.init();
    double accWl = 0.0;                                     // this lane's W_t column (fast path)
    constexpr bool query = QRY != 0;                        // posterior queries: generic path

    int64_t tile = blockIdx.x;
    int buf = 0;
    float rs_next = 1.0f;                                   // next tile's row scale (tid < BM)
    if (tile < ntiles) {
        dma_issue_tile(A, tile, BM, smem, LY.RS);
        const int64_t r0 = A.row_begin + tile * BM;
        if (tid < BM && r0 + tid < A.row_end && A.rowscale) rs_next = A.rowscale[r0 + tid];
    }
    for (; tile < ntiles; tile += gridDim.x, buf ^= 1) {
        const int64_t r0 = A.row_begin + tile * BM;
        const int rows = (int)((A.row_end - r0) < BM ? (A.row_end - r0) : BM);
        uint8_t *Vs = smem + (buf ? LY.off_v1 : 0);
        const float rs = rs_next;
        __builtin_amdgcn_s_waitcnt(0);                      // this tile's copy has landed
        __syncthreads();                                    // ... for every wave; old tile done
        if (tile + gridDim.x < ntiles) {
            const int64_t rn = A.row_begin + (tile + gridDim.x) * BM;
            dma_issue_tile(A, tile + gridDim.x, BM, smem + (buf ? 0 : LY.off_v1), LY.RS);
            if (tid < BM && rn + tid < A.row_end && A.rowscale) rs_next = A.rowscale[rn + tid];
        }
        if (tid < BM) {
            const float u = tid < rows ? rs : 1.0f;
            rowf[tid] = (float)A.coef * u * tsc;
            rowu[tid] = u;
        }

        // ---- a3: partial correlations over this wave's K-slice
        f32x4 c4[MS][NT];
#pragma unroll
        for (int m = 0; m < MS; ++m)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) c4[m][nt] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KSS; ++ks) {
            const int kstep = wave * KSS + ks;
#pragma unroll
            for (int m = 0; m < MS; ++m) {
                const uint8_t *arow = Vs + (m * 16 + rl) * LY.RS + kstep * 64 + g * 16;
                const u32x4 ah = *(const u32x4 *)arow;
                if constexpr (P == P_BF16X3) {
                    const u32x4 al = *(const u32x4 *)(arow + 2 * A.Dp);
                    const bf16x8 AH = __builtin_bit_cast(bf16x8, ah);
                    const bf16x8 AL = __builtin_bit_cast(bf16x8, al);
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) {
                        c4[m][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            AH, __builtin_bit_cast(bf16x8, treg[ks][nt][1]), c4[m][nt], 0, 0, 0);
                        c4[m][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            AL, __builtin_bit_cast(bf16x8, treg[ks][nt][0]), c4[m][nt], 0, 0, 0);
                        c4[m][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            AH, __builtin_bit_cast(bf16x8, treg[ks][nt][0]), c4[m][nt], 0, 0, 0);
                    }
                } else if constexpr (P == P_F16) {
                    const f16x8 AH = __builtin_bit_cast(f16x8, ah);
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) {
                        c4[m][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                            AH, __builtin_bit_cast(f16x8, treg[ks][nt][1]), c4[m][nt], 0, 0, 0);
                        c4[m][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                            AH, __builtin_bit_cast(f16x8, treg[ks][nt][0]), c4[m][nt], 0, 0, 0);
                    }
                } else {
                    const bf16x8 AH = __builtin_bit_cast(bf16x8, ah);
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) {
                        c4[m][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            AH, __builtin_bit_cast(bf16x8, treg[ks][nt][1]), c4[m][nt], 0, 0, 0);
                        c4[m][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            AH, __builtin_bit_cast(bf16x8, treg[ks][nt][0]), c4[m][nt], 0, 0, 0);
                    }
                }
            }
        }
        // ---- fixed-order sum of the eight K-slices: slot k = slice k + slice k+4
        if (wave >= 4) {
#pragma unroll
            for (int m = 0; m < MS; ++m)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    red[(((wave - 4) * MS + m) * NT + nt) * 64 + lane] = c4[m][nt];
        }
        lds_barrier();
        if (wave < 4) {
#pragma unroll
            for (int m = 0; m < MS; ++m)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    f32x4 *slot = &red[((wave * MS + m) * NT + nt) * 64 + lane];
                    *slot = c4[m][nt] + *slot;
                }
        }
        lds_barrier();
        if constexpr (!query) {
            ks_post<P, BM, NT, DPT, KG>(A, LY, Vs, red, Cs, Us, rowf, rowu, lrs, r0, rows, acc,
                                         accWl, ereg, uact, ucol);
            continue;
        }
        for (int o = tid; o < BM * A.Wp; o += kThreads) {
            const int row = o / A.Wp, col = o - row * A.Wp;
            const int m = row >> 4, rr = row & 15, nt = col >> 4;
            const int ln = (rr >> 2) * 16 + (col & 15), q = rr & 3;
            float v = red[((0 * MS + m) * NT + nt) * 64 + ln][q];
            v += red[((1 * MS + m) * NT + nt) * 64 + ln][q];
            v += red[((2 * MS + m) * NT + nt) * 64 + ln][q];
            v += red[((3 * MS + m) * NT + nt) * 64 + ln][q];
            Cs[row * LY.CSW + col] = v * rowf[row] + lrs[col];
        }
        lds_barrier();
        if constexpr (query)
            tile_post<P, BM, DPT, KG>(A, PL, Vs, Cs, Us, rowu, lrs, r0, rows, acc, ereg, uact,
                                      ucol);
    }
    if constexpr (!query) {
        // the per-lane W_t columns of the eight waves, summed in wave order
        __syncthreads();
        double *wsh = (double *)(smem + LY.off_red);
        wsh[wave * 64 + lane] = accWl;
        __syncthreads();
        acc.W[0] = acc.W[1] = 0.0;
        if (tid < 64) {
            double t = 0.0;
            for (int k = 0; k < kThreads / 64; ++k) t += wsh[k * 64 + tid];
            acc.W[0] = t;
        }
    }
    if (A.partials) write_partials(A, acc, smem);
}

// ------------------------------------------------------------------------------------------
// Wide-row E(+M) pass, for rows too long to double-buffer a tile of them in LDS (D = 2048 in
// fp16 is 8 KiB per row).  A tile is kWideBM = 128 rows.  The eight waves are 4 window groups x
// 2 K-halves: wave (iw, kh) accumulates the window tiles iw, iw + 4, .. (NTW of them) for all 8
// row blocks of the tile over its half of the 2D reals.  The product is formed transposed
// (template fragments as the A operand, observation fragments as B), so the accumulators come
// out with one observation row per lane column.  The row tile streams through a ring of
// kWideSlots LDS slots (kWideKSS k-steps of each half per slot) by direct global-to-LDS copies;
// template fragments stream from L2 one slot ahead.  Every wave issues the same number of vector
// memory loads per slot (out-of-range k-steps and window tiles load a valid dummy address), so
// a fixed s_waitcnt count makes slot s resident while slots s+1, s+2 stay in flight.  The two
// K-halves are summed through the C tile in LDS (a two-term sum, so the order cannot change
// it); then the posteriors (tile_rows), W_t, and U = w E and the M-step in chunks of UR rows,
// the M-step reading the tile's rows again from global memory.

constexpr int kWideSlots = 3;
constexpr int kWideKSS = 2;

struct WideLds {
    int CSW, slot_bytes, off_u, off_f, off_lr, off_s, total;
};
__host__ __device__ inline WideLds wide_lds(int K, int Wp, int NTW, int UR) {
    WideLds l;
    // 64 NTW columns (the window tiles of all wave groups; those past Wp are zero), float4
    // rows, conflict-free columns
    l.CSW = 64 * NTW + 4;
    l.slot_bytes = 2 * kWideKSS * kWideBM * 64;        // [half][k-step][row][64 B]
    const int ring = kWideSlots * l.slot_bytes;
    l.off_u = align_up(kWideBM * l.CSW * 4, 16);
    const int post = l.off_u + UR * K * 8;
    l.off_f = align_up(ring > post ? ring : post, 16);
    l.off_lr = l.off_f + 2 * kWideBM * 4;
    l.off_s = align_up(l.off_lr + Wp * 4, 16);
    l.total = l.off_s + kMaxD * 16;                    // FP64 M-step sums, kept across tiles
    return l;
}

// s_waitcnt with only the vector-memory count constrained (gfx9 encoding), then a compiler
// barrier so no memory access moves across it.
template <int N>
__device__ __forceinline__ void wait_vm() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
    asm volatile("" ::: "memory");
}


typedef __amdgpu_buffer_rsrc_t rsrc_t;
__device__ __forceinline__ rsrc_t make_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                             0x00020000);
}

// Slot s of the tile behind rsrc V: k-steps half_base + s KSS + ss of its 128 rows; wave w copies
// row block w of both halves and both k-steps (4 copies of 1 KiB).  voff = this lane's byte
// offset (row, clamped to the tile, and 16-byte piece); k-steps past the end copy a valid
// stand-in that is never used.
__device__ __forceinline__ void wide_dma(rsrc_t V, uint32_t voff, int s, int KS, int KH0,
                                         uint8_t *slot) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int ss = 0; ss < kWideKSS; ++ss) {
            int ks = (h ? KH0 : 0) + s * kWideKSS + ss;
            ks = ks < KS ? ks : KS - 1;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(
                V,
                (__attribute__((address_space(3))) void *)(slot + ((h * kWideKSS + ss) * kWideBM +
                                                                   16 * wave) * 64),
                16, voff, (uint32_t)ks * 64u, 0, 0);
        }
}

// Template fragments of k-step ks (clamped into [0, ke)) for this wave's window tiles; toff[n]
// is the byte offset of tile n's fragment column for this lane.
template <int NTW>
__device__ __forceinline__ void wide_tload(rsrc_t Th, rsrc_t Tl, const uint32_t (&toff)[NTW],
                                           int ks, int ke, u32x4 (&th)[NTW], u32x4 (&tl)[NTW]) {
    int k = ks < ke ? ks : ke - 1;
    k = k < 0 ? 0 : k;
    const uint32_t so = (uint32_t)k * 1024u;
#pragma unroll
    for (int n = 0; n < NTW; ++n) {
        th[n] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(Th, toff[n], so, 0));
        tl[n] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(Tl, toff[n], so, 0));
    }
}

// U (UR rows) = w . [Re E | Im E] on FP32 matrix cores with this wave's B fragments in
// registers: wave w computes U columns 16 w .. 16 w + 15 over KGM k-steps of 4 columns of Cs
// (columns past the window are zero).
template <int UR, int KGM>
__device__ __forceinline__ void u_wide_reg(const float *Cs, int CSW, const float (&ereg)[KGM],
                                           int K, const float *rowu, float2 *Us, int ucol) {
    constexpr int MS = UR / 16;
    const int lane = threadIdx.x & 63, g = lane >> 4, rl = lane & 15;
    if ((ucol & ~15) >= 2 * K) return;             // this wave's U column tile is past 2K
    f32x4 acc[MS];
#pragma unroll
    for (int m = 0; m < MS; ++m) acc[m] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < KGM; ++kk)
#pragma unroll
        for (int m = 0; m < MS; ++m) {
            const float a = Cs[(m * 16 + rl) * CSW + kk * 4 + g];
            acc[m] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, ereg[kk], acc[m], 0, 0, 0);
        }
    if (ucol < 2 * K) {
#pragma unroll
        for (int m = 0; m < MS; ++m)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = m * 16 + 4 * g + q;
                const float v = acc[m][q] * rowu[row];
                if (ucol < K)
                    Us[row * K + ucol].x = v;
                else
                    Us[row * K + ucol - K].y = v;
            }
    }
}

template <int P, int NTW, int UR>
__global__ __launch_bounds__(kThreads) void pass_wide_kernel(PassArgs A) {
    static_assert(P == P_F16 || P == P_BF16, "one 16-bit observation plane");
    constexpr int BM = kWideBM, MJ = BM / 16, DPT = kMaxDPerThread;
    constexpr int NTL = kWideKSS * NTW * 2;            // template loads per wave per slot
    constexpr int NDL = 2 * kWideKSS;                  // LDS copies per wave per slot

    if ((A.flags & PF_CHECK_STOP) && *A.stopped) return;

    extern __shared__ __align__(16) uint8_t smem[];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform, in an SGPR
    const int g = lane >> 4, c = lane & 15;
    const WideLds LY = wide_lds(A.K, A.Wp, NTW, UR);
    float *Cs = (float *)smem;
    float2 *Us = (float2 *)(smem + LY.off_u);
    float *rowf = (float *)(smem + LY.off_f);
    float *rowu = rowf + BM;
    float *lrs = (float *)(smem + LY.off_lr);
    double2 *Sacc = (double2 *)(smem + LY.off_s);      // thread t owns entries t, t + 512, ..
    for (int i = tid; i < A.Wp; i += kThreads) lrs[i] = A.logrho32[i];
    for (int d = tid; d < kMaxD; d += kThreads) Sacc[d] = make_double2(0.0, 0.0);
    const float tsc = *A.tscale;

    const int NT = A.Wp / 16, KS = A.Dp / 32;
    const int KH0 = (KS + 1) / 2;
    const int NS = (KH0 + kWideKSS - 1) / kWideKSS;
    const int iw = wave & 3, kh = wave >> 2;
    const int kb = kh ? KH0 : 0, ke = kh ? KS : KH0;
    const uint32_t tbytes = (uint32_t)NT * KS * 1024u;
    const rsrc_t Th = make_rsrc(A.Thi, tbytes), Tl = make_rsrc(A.Tlo, tbytes);
    uint32_t toff[NTW];
#pragma unroll
    for (int n = 0; n < NTW; ++n) {
        const int nt = iw + 4 * n < NT ? iw + 4 * n : 0;
        toff[n] = ((uint32_t)nt * KS * 64u + lane) * 16u;
    }

    PassAcc<DPT> acc;
    acc.init();
    const int64_t ntiles = (A.row_end - A.row_begin + BM - 1) / BM;
    float rs_next = 1.0f;
    int64_t tile = blockIdx.x;
    if (tile < ntiles) {
        const int64_t r0 = A.row_begin + tile * BM;
        if (tid < BM && r0 + tid < A.row_end && A.rowscale) rs_next = A.rowscale[r0 + tid];
    }
    for (; tile < ntiles; tile += gridDim.x) {
        const int64_t r0 = A.row_begin + tile * BM;
        const int rows = (int)((A.row_end - r0) < BM ? (A.row_end - r0) : BM);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();                               // the previous tile's post phase is done
        if (tid < BM) {
            const float u = tid < rows ? rs_next : 1.0f;
            rowf[tid] = (float)A.coef * u * tsc;
            rowu[tid] = u;
        }

        // ---- a3: this wave's window tiles over its K-half, slot by slot
        f32x4 ac[NTW][MJ];
#pragma unroll
        for (int n = 0; n < NTW; ++n)
#pragma unroll
            for (int m = 0; m < MJ; ++m) ac[n][m] = (f32x4){0.f, 0.f, 0.f, 0.f};
        u32x4 th[kWideKSS][NTW], tl[kWideKSS][NTW];
        const rsrc_t Vt = make_rsrc(A.V + r0 * A.rowbytes, (uint32_t)(rows * A.rowbytes));
        uint32_t voff;
        {
            const int row = 16 * wave + (lane >> 2);
            voff = (uint32_t)((row < rows ? row : rows - 1) * A.rowbytes) + (lane & 3) * 16u;
        }
        // Every slot step issues the same loads (stand-ins past the end, copied into slots that
        // are free), so the loop body is the same on every trip and slot s is resident once at
        // most the last NTL + NDL loads of this wave are outstanding.
        wide_dma(Vt, voff, 0, KS, KH0, smem);
        asm volatile("" ::: "memory");                 // keep the steady-state issue order
#pragma unroll
        for (int ss = 0; ss < kWideKSS; ++ss)
            wide_tload<NTW>(Th, Tl, toff, kb + ss, ke, th[ss], tl[ss]);
        asm volatile("" ::: "memory");
        wide_dma(Vt, voff, 1, KS, KH0, smem + LY.slot_bytes);
        for (int s = 0; s < NS; ++s) {
            wait_vm<NTL + NDL>();
            lds_barrier();
            const uint8_t *slot = smem + (s % kWideSlots) * LY.slot_bytes;
#pragma unroll
            for (int ss = 0; ss < kWideKSS; ++ss) {
                const int ks = kb + s * kWideKSS + ss;
                if (ks < ke) {
#pragma unroll
                    for (int m = 0; m < MJ; ++m) {
                        const u32x4 vf = *(const u32x4 *)(slot + ((kh * kWideKSS + ss) * BM +
                                                                  16 * m + c) * 64 + g * 16);
#pragma unroll
                        for (int n = 0; n < NTW; ++n) {
                            // (a tile past the window's end multiplies a stand-in fragment;
                            // its accumulator is never stored)
                            if constexpr (P == P_F16) {
                                const f16x8 V8 = __builtin_bit_cast(f16x8, vf);
                                ac[n][m] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                                    __builtin_bit_cast(f16x8, tl[ss][n]), V8, ac[n][m], 0, 0, 0);
                                ac[n][m] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                                    __builtin_bit_cast(f16x8, th[ss][n]), V8, ac[n][m], 0, 0, 0);
                            } else {
                                const bf16x8 V8 = __builtin_bit_cast(bf16x8, vf);
                                ac[n][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                    __builtin_bit_cast(bf16x8, tl[ss][n]), V8, ac[n][m], 0, 0, 0);
                                ac[n][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                    __builtin_bit_cast(bf16x8, th[ss][n]), V8, ac[n][m], 0, 0, 0);
                            }
                        }
                    }
                }
                wide_tload<NTW>(Th, Tl, toff, kb + (s + 1) * kWideKSS + ss, ke, th[ss], tl[ss]);
            }
            asm volatile("" ::: "memory");
            wide_dma(Vt, voff, s + 2, KS, KH0, smem + ((s + 2) % kWideSlots) * LY.slot_bytes);
        }

        // ---- the two K-halves summed into the C tile (which overlays the ring), then
        // l' = coef C + log rho; next tile's row scale
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (kh == 0) {
#pragma unroll
            for (int n = 0; n < NTW; ++n) {
                const int nt = iw + 4 * n;
                if (nt >= NT) continue;
#pragma unroll
                for (int m = 0; m < MJ; ++m)
                    *(f32x4 *)(Cs + (16 * m + c) * LY.CSW + 16 * nt + 4 * g) = ac[n][m];
            }
        }
        __syncthreads();
        if (kh == 1) {
#pragma unroll
            for (int n = 0; n < NTW; ++n) {
                const int nt = iw + 4 * n;
                if (nt >= NT) {                        // zero columns past the window tiles
#pragma unroll
                    for (int m = 0; m < MJ; ++m)
                        *(f32x4 *)(Cs + (16 * m + c) * LY.CSW + 16 * nt + 4 * g) =
                            (f32x4){0.f, 0.f, 0.f, 0.f};
                    continue;
                }
                const f32x4 lr4 = *(const f32x4 *)(lrs + 16 * nt + 4 * g);
#pragma unroll
                for (int m = 0; m < MJ; ++m) {
                    f32x4 *p = (f32x4 *)(Cs + (16 * m + c) * LY.CSW + 16 * nt + 4 * g);
                    const float rf = rowf[16 * m + c];
                    const f32x4 o = *p;
                    f32x4 l;
#pragma unroll
                    for (int q = 0; q < 4; ++q) l[q] = (o[q] + ac[n][m][q]) * rf + lr4[q];
                    *p = l;
                }
            }
        }
        if (tile + gridDim.x < ntiles) {
            const int64_t rn = A.row_begin + (tile + gridDim.x) * BM;
            if (tid < BM && rn + tid < A.row_end && A.rowscale) rs_next = A.rowscale[rn + tid];
        }
        __syncthreads();

        // ---- a4 + a5
        tile_rows<P, BM, DPT>(A, LY.CSW, Cs, lrs, r0, rows, acc);
        if (!(A.flags & PF_ACC_M)) continue;
        __syncthreads();
        tile_wsum<P, DPT>(A, LY.CSW, Cs, rows, acc);
        // B fragments of U = w [Re E | Im E] for this wave's 16-column tile of U, in registers
        // for the whole tile (one column tile per wave when 2K <= 128)
        const bool ureg = 2 * A.K <= 16 * (kThreads / 64);
        const int ucol = wave * 16 + c;
        constexpr int KGM = 16 * NTW;                  // 4-column k-steps over 64 NTW columns
        float ereg[KGM];
        if (ureg) {
            // E2 row 4 kk + g, column ucol; rows past Wp are clamped (they meet zero
            // posteriors) and so are columns past 2K (their U columns are not stored)
            const rsrc_t Er = make_rsrc(A.E2, (uint32_t)(A.Wp * 2 * A.K * 4));
            const int ccol = ucol < 2 * A.K ? ucol : 2 * A.K - 1;
#pragma unroll
            for (int kk = 0; kk < KGM; ++kk) {
                const int row = 4 * kk + g < A.Wp ? 4 * kk + g : A.Wp - 1;
                ereg[kk] = __builtin_bit_cast(
                    float, __builtin_amdgcn_raw_buffer_load_b32(
                               Er, (uint32_t)(row * 2 * A.K + ccol) * 4u, 0u, 0));
            }
        }
        for (int rc = 0; rc < rows; rc += UR) {
            if (rc) __syncthreads();                   // the previous chunk's U is consumed
            if (ureg)
                u_wide_reg<UR, KGM>(Cs + rc * LY.CSW, LY.CSW, ereg, A.K, rowu + rc, Us, ucol);
            else
                u_mfma<UR>(Cs + rc * LY.CSW, LY.CSW, A.E2, A.Wp, A.K, rowu + rc, Us);
            __syncthreads();
            const int nr = rows - rc < UR ? rows - rc : UR;
            const uint8_t *vb = A.V + (r0 + rc) * A.rowbytes;
            // M-step: thread t owns the four entries 4t .. 4t+3 (16 bytes of every row), with
            // 8 rows of loads in flight
            const int d0 = 4 * tid;
            if (d0 < A.D) {
                const int k0 = d0 / A.Q, k3 = (d0 + 3) / A.Q;
                float sr[4] = {0.f, 0.f, 0.f, 0.f}, si[4] = {0.f, 0.f, 0.f, 0.f};
                for (int j0 = 0; j0 < nr; j0 += 8) {
                    u32x4 raw[8];
#pragma unroll
                    for (int t = 0; t < 8; ++t) {
                        const int j = j0 + t < nr ? j0 + t : nr - 1;
                        raw[t] = *(const u32x4 *)(vb + (int64_t)j * A.rowbytes + 16 * tid);
                    }
#pragma unroll
                    for (int t = 0; t < 8; ++t) {
                        if (j0 + t >= nr) break;
                        const float2 *ur = Us + (j0 + t) * A.K;
                        float2 u[4];
                        u[0] = ur[k0];
                        if (k3 == k0) {
                            u[1] = u[2] = u[3] = u[0];
                        } else {
#pragma unroll
                            for (int e = 1; e < 4; ++e) u[e] = ur[(d0 + e) / A.Q];
                        }
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            float vr, vi;
                            if constexpr (P == P_F16) {
                                const _Float16 *h = (const _Float16 *)&raw[t];
                                vr = (float)h[2 * e];
                                vi = (float)h[2 * e + 1];
                            } else {
                                const __bf16 *h = (const __bf16 *)&raw[t];
                                vr = (float)h[2 * e];
                                vi = (float)h[2 * e + 1];
                            }
                            sr[e] += u[e].x * vr - u[e].y * vi;
                            si[e] += u[e].x * vi + u[e].y * vr;
                        }
                    }
                }
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (d0 + e < A.D) {
                        Sacc[d0 + e].x += (double)sr[e];
                        Sacc[d0 + e].y += (double)si[e];
                    }
            }
        }
    }
    __syncthreads();                                   // Sacc rows were written by other waves
#pragma unroll
    for (int cc = 0; cc < DPT; ++cc) acc.S[cc] = Sacc[tid + cc * kThreads];
    __syncthreads();
    if (A.partials) write_partials(A, acc, smem);
}

// ------------------------------------------------------------------------------------------
// Row-stream correlation pass (the contraction against the W rotated templates, as the method
// states it) for one 16-bit plane of observations with D = 512 and windows up to 64, built so
// that its row tiles stream at HBM rate: one workgroup per CU, 16-row tiles copied global-to-LDS
// two tiles ahead of their use (three LDS buffers, completion tracked by exact vector-memory
// counts), and two workgroup barriers per tile.
//   * K-split: wave w owns k-steps 4w .. 4w + 3 (reals 128 w .. 128 w + 127) and holds the
//     template rows of its slice for every window tile in registers (hi + lo, built once per
//     launch from a_t); per tile it reads its slice of the 16 rows from LDS once (MFMA A
//     fragments) and keeps it in registers for the M-step.
//   * The eight partial correlations go to LDS; wave w then sums them in wave order for rows
//     2 w and 2 w + 1 (32 lanes per row, two window columns per lane), forms the prior-weighted
//     log-sum-exp and the posteriors with 32-lane reductions, and writes the posteriors as 16-bit
//     hi + lo planes.
//   * U = w E is formed transposed and per wave, for the angular frequencies of the wave's own
//     entries only (U^T = E'^T w^T: three 16x16x32 products, E' hi + lo in registers), and left
//     in a wave-private LDS block; the M-step then runs on the wave's own row fragments, so no
//     row is read from LDS twice and no U is shared between waves.  Per-lane FP32 sums over the
//     lane's rows are folded into FP64 every kKrFlush tiles (16-lane DPP sums, then each lane
//     keeps two of its group's 32 values).
// Needs Dp = 1024 (D = 512 with Q in {8, 16, 32, 64}: a lane's four entries of a k-step share
// one frequency and a wave's entries span at most eight) and Wp = 16 NT <= 64.

constexpr int kKrBM = 16;                 // rows per tile
constexpr int kKrBufs = 3;                // LDS row-tile buffers (two tiles in flight)
constexpr int kKrFlush = 16;              // tiles between FP32 -> FP64 folds of the M-step sums
constexpr int kKrWS = 144;                // bytes per posterior row of one 16-bit plane (64 + pad)
constexpr int kKrUS = 20;                 // floats per row of a wave's U block (16 + pad)
// Partial-correlation slots (16 B each) per (wave, window tile): lane 16 g + j's slot is 17 g + j,
// so that both the MFMA-order writes and the row-order reads are free of bank conflicts.
constexpr int kKrRedTile = 68;

struct KrLds {
    int RS, off_red, off_w, off_up, off_rs, off_lr, off_wacc, total;
};
__host__ __device__ inline KrLds kr_lds(int Dp) {
    KrLds l;
    l.RS = 2 * Dp + 16;                                   // staged row, padded
    l.off_red = align_up(kKrBufs * kKrBM * l.RS, 16);     // 8 waves x 4 tiles x 64 lanes x 16 B
    l.off_w = l.off_red + 8 * 4 * kKrRedTile * 16;
    l.off_up = l.off_w + 2 * kKrBM * kKrWS;               // hi plane, then lo plane
    l.off_rs = l.off_up + 8 * 16 * kKrUS * 4;             // per-wave U blocks
    l.off_lr = l.off_rs + 4 * 64 * 4;                     // row scales of four tiles
    l.off_wacc = l.off_lr + 64 * 4;                       // FP64 W_t sums: 16 row lanes x 64
    l.total = l.off_wacc + 16 * 64 * 8;
    return l;
}

template <int P, int NT, int QRY>
__global__ __launch_bounds__(kThreads) void pass_kr_kernel(PassArgs A) {
    static_assert(P == P_F16 || P == P_BF16, "one 16-bit plane");
    static_assert(NT >= 1 && NT <= 4, "windows up to 64");
    typedef typename std::conditional<P == P_F16, _Float16, __bf16>::type H;
    typedef typename std::conditional<P == P_F16, f16x8, bf16x8>::type H8;
    constexpr int KSS = 4, BM = kKrBM;
    constexpr bool query = QRY != 0;
    if ((A.flags & PF_CHECK_STOP) && *A.stopped) return;

    extern __shared__ __align__(16) uint8_t smem[];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int g = lane >> 4, rl = lane & 15;
    const KrLds LY = kr_lds(A.Dp);
    f32x4 *red = (f32x4 *)(smem + LY.off_red);
    uint8_t *wsh = smem + LY.off_w;
    float *up = (float *)(smem + LY.off_up) + wave * 16 * kKrUS;
    float *rsb = (float *)(smem + LY.off_rs);
    float *lrs = (float *)(smem + LY.off_lr);
    const int D = A.D, K = A.K, Q = A.Q, W = A.W, Wp = A.Wp;
    const bool accm = (A.flags & PF_ACC_M) != 0;
    // exact vector-memory counts hold only while the loop issues nothing but its tile copies
    const bool deep = !(A.flags & (PF_STORE_LSE | PF_LOAD_LSE | PF_QUERY));

    for (int i = tid; i < 64; i += kThreads) lrs[i] = i < Wp ? A.logrho32[i] : -INFINITY;
    // a_t and the phase rows staged in LDS (where the third row buffer and the partials go,
    // first written after the barrier that ends the prologue); the template scale from
    // max |Re a|, |Im a| (a power of two, as in the other 16-bit passes)
    uint8_t *stg = smem + 2 * BM * LY.RS;
    const double amax = stage_a_e2(A, stg, (double *)(smem + LY.off_up));
    const float2 *as = (const float2 *)stg;
    const float *es = (const float *)(stg + 8 * D);
    const int qs = __builtin_ctz(Q);                   // Q is a power of two
    float sc = 1.0f, tsc = 1.0f;
    if (amax > 0.0) {
        const int e = ilogb(amax);
        sc = ldexpf(1.0f, scale_target(P) - e);
        tsc = ldexpf(1.0f, e - scale_target(P));
    }
    // this wave's template slice: T[r][i] = (Re, Im)(a_d exp(-i k_d theta_i)) sc, d = r / 2,
    // B fragments (column i = 16 nt + lane % 16, reals 8 g .. 8 g + 7 of the k-step), hi + lo
    u32x4 treg[KSS][NT][2];
    // (the lane's four entries of a k-step share one frequency, Q >= 8; sc, a power of two, is
    // applied to a first, which leaves every product as it would be scaled afterwards)
#pragma unroll
    for (int ks = 0; ks < KSS; ++ks) {
        const int d0 = ((wave * KSS + ks) * 32 + 8 * g) >> 1;       // a multiple of 4, < D
        const int k = d0 >> qs;
        const float4 a01 = *(const float4 *)(as + d0), a23 = *(const float4 *)(as + d0 + 2);
        const float ar[4] = {a01.x * sc, a01.z * sc, a23.x * sc, a23.z * sc};
        const float ai[4] = {a01.y * sc, a01.w * sc, a23.y * sc, a23.w * sc};
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const float *Ei = es + (nt * 16 + rl) * 2 * K;
            tpl_frag4<H>(ar, ai, Ei[k], Ei[K + k], treg[ks][nt][0], treg[ks][nt][1]);
        }
    }
    // A fragments of U^T = E'^T w^T: row m of E'^T is Re (m even) or Im (m odd) of
    // exp(+i k theta_i) at k = kbase + m / 2, the frequencies of this wave's entries
    const int kbase = (64 * wave) / Q, nk = 64 / Q;
    H8 eh[2], el[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        H hv[8], lv[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int i = 32 * s + 8 * g + t, k = kbase + (rl >> 1);
            const bool ok = i < Wp && (rl >> 1) < nk && k < K;
            const float v = es[(ok ? i * 2 * K + ((rl & 1) ? K : 0) + k : 0)];
            const float x = ok ? v : 0.f;
            hv[t] = (H)x;
            lv[t] = (H)(x - (float)hv[t]);
        }
        eh[s] = __builtin_bit_cast(H8, hv);
        el[s] = __builtin_bit_cast(H8, lv);
    }
    // the U column (2 (k - kbase)) each of this lane's k-steps needs
    int um[KSS];
#pragma unroll
    for (int ks = 0; ks < KSS; ++ks) um[ks] = 2 * ((16 * (wave * KSS + ks) + 4 * g) / Q - kbase);

    const int64_t ntiles = (A.row_end - A.row_begin + BM - 1) / BM;
    const int64_t nmine = ntiles > (int64_t)blockIdx.x
                              ? (ntiles - 1 - (int64_t)blockIdx.x) / gridDim.x + 1 : 0;
    // copy of this workgroup's j-th tile into buffer j % 3: 32 chunks of 1 KiB (wave w: chunks w,
    // w + 8, w + 16, w + 24, i.e. rows w / 2 + 4 cc, half w % 2; rows past the end repeat the last
    // row, so every tile issues the same number of copies), and wave 0 the 64 row scales at and
    // after the tile's first row into slot j % 4
    const int64_t tstride = (int64_t)gridDim.x * BM;
    auto issue = [&](int j) {
        const int64_t r0 = A.row_begin + (int64_t)blockIdx.x * BM + (int64_t)j * tstride;
        uint8_t *buf = smem + (j % kKrBufs) * BM * LY.RS;
        const int rc = wave >> 1, kc = wave & 1;
        if (r0 + BM <= A.row_end) {
            const uint8_t *src = A.V + (r0 + rc) * A.rowbytes + kc * 1024 + lane * 16;
#pragma unroll
            for (int cc = 0; cc < 4; ++cc)
                dma_to_lds<16>(src + (int64_t)(4 * cc) * A.rowbytes,
                               buf + (rc + 4 * cc) * LY.RS + kc * 1024);
        } else {
#pragma unroll
            for (int cc = 0; cc < 4; ++cc) {
                const int r = rc + 4 * cc;
                const int64_t row = r0 + r < A.row_end ? r0 + r : A.row_end - 1;
                dma_to_lds<16>(A.V + row * A.rowbytes + kc * 1024 + lane * 16,
                               buf + r * LY.RS + kc * 1024);
            }
        }
        if (wave == 0) {
            const int64_t row = r0 + lane < A.row_end ? r0 + lane : A.row_end - 1;
            dma_to_lds<4>(A.rowscale + row, rsb + (j & 3) * 64);
        }
    };

    // posteriors: every wave takes two rows, 32 lanes per row; this lane's two window columns
    // 2 px .. 2 px + 1 (half ph of the partial slot of window tile pnt, lane group pg); the row
    // factor; W_t of the two columns (FP32 over 16 tiles, then added into FP64 sums in LDS that
    // only this thread touches)
    const int px = lane & 31, pnt = px >> 3, pg = (px >> 1) & 3, ph = px & 1;
    const float ct = (float)A.coef * tsc;
    float accW[2] = {0.f, 0.f};
    double *wacc = (double *)(smem + LY.off_wacc) + (2 * wave + (lane >> 5)) * 64 + 2 * px;
    wacc[0] = wacc[1] = 0.0;
    int nfw = 0;
    float sr[KSS][4], si[KSS][4];                // M-step sums of this lane's rows (FP32)
#pragma unroll
    for (int ks = 0; ks < KSS; ++ks)
#pragma unroll
        for (int e = 0; e < 4; ++e) sr[ks][e] = si[ks][e] = 0.f;
    double s64[2] = {0.0, 0.0};                  // two of the lane group's 32 values, FP64
    double acc_lse = 0.0, acc_wc = 0.0, acc_rows = 0.0;
    int nfl = 0;
    // fold the FP32 M-step sums into FP64: sum over the 16 lanes of the group (its 16 rows of
    // every tile), then lane rl keeps values rl and rl + 16 of the group's 32
    auto fold = [&]() {
        float x0 = 0.f, x1 = 0.f;
#pragma unroll
        for (int ks = 0; ks < KSS; ++ks)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float a = row16_sum(sr[ks][e]), b = row16_sum(si[ks][e]);
                const int i = ks * 8 + e * 2;
                x0 = rl == i ? a : x0;
                x0 = rl == i + 1 ? b : x0;
                x1 = rl + 16 == i ? a : x1;
                x1 = rl + 16 == i + 1 ? b : x1;
                sr[ks][e] = si[ks][e] = 0.f;
            }
        s64[0] += (double)x0;
        s64[1] += (double)x1;
    };

    // ---- a3: this wave's K-slice of the correlations of the tile in buffer bt (formed
    // transposed, template fragments as the A operand: lane 16 g + j ends with row j, columns
    // 16 nt + 4 g .. 16 nt + 4 g + 3)
    f32x4 c4[NT];
    auto products = [&](int bt) {
        const uint8_t *Vs = smem + bt * BM * LY.RS;
        u32x4 af[KSS];
#pragma unroll
        for (int ks = 0; ks < KSS; ++ks)
            af[ks] = *(const u32x4 *)(Vs + rl * LY.RS + (wave * KSS + ks) * 64 + g * 16);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) c4[nt] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KSS; ++ks) {
            const H8 bv = __builtin_bit_cast(H8, af[ks]);
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                if constexpr (P == P_F16) {
                    c4[nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                        __builtin_bit_cast(H8, treg[ks][nt][1]), bv, c4[nt], 0, 0, 0);
                    c4[nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                        __builtin_bit_cast(H8, treg[ks][nt][0]), bv, c4[nt], 0, 0, 0);
                } else {
                    c4[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        __builtin_bit_cast(H8, treg[ks][nt][1]), bv, c4[nt], 0, 0, 0);
                    c4[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        __builtin_bit_cast(H8, treg[ks][nt][0]), bv, c4[nt], 0, 0, 0);
                }
            }
        }
    };
    auto put_red = [&]() {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
            red[(wave * 4 + nt) * kKrRedTile + 17 * g + rl] = c4[nt];
    };

    // ---- a4: rows 2 wave, 2 wave + 1 of tile j, 32 lanes per row, columns 2 x, 2 x + 1 per
    // lane (x = lane % 32): the 8 partial sums in wave order, the log-sum-exp by 32-lane
    // reductions (16-lane DPP rows, then the swizzle across the pair of rows), the posteriors
    // written as 16-bit hi + lo planes
    auto posteriors = [&](int64_t r0, int rows, const float *rsv) {
        const int r = 2 * wave + (lane >> 5);
        const bool rv = r < rows;
        float l[2], e[2];
        const float2 lr2 = *(const float2 *)(lrs + 2 * px);
        const bool cok[2] = {2 * px < W, 2 * px + 1 < W};
        {
            const float *rp = (const float *)red + 4 * (pnt * kKrRedTile + 17 * pg + r) + 2 * ph;
            float2 v = *(const float2 *)rp;
#pragma unroll
            for (int w2 = 1; w2 < 8; ++w2) {
                const float2 t = *(const float2 *)(rp + 4 * (w2 * 4 * kKrRedTile));
                v.x += t.x;
                v.y += t.y;
            }
            const float rf = ct * rsv[r];
            l[0] = (rv && cok[0]) ? v.x * rf + lr2.x : -INFINITY;
            l[1] = (rv && cok[1]) ? v.y * rf + lr2.y : -INFINITY;
        }
        float lse;
        if (A.flags & PF_LOAD_LSE) {
            lse = rv ? (float)A.lse[r0 + r] : 0.f;
#pragma unroll
            for (int q = 0; q < 2; ++q) e[q] = __expf(l[q] - lse);
        } else {
            float mx = row16_max(fmaxf(l[0], l[1]));
            mx = fmaxf(mx, swz_xor16(mx));
            if (!rv) mx = 0.f;                         // (an empty row: every l is -inf)
#pragma unroll
            for (int q = 0; q < 2; ++q) e[q] = __expf(l[q] - mx);   // exp(-inf) = 0
            float sx = row16_sum(e[0] + e[1]);
            sx += swz_xor16(sx);
            lse = mx + __logf(sx);
            const float is = rv ? __builtin_amdgcn_rcpf(sx) : 0.f;
#pragma unroll
            for (int q = 0; q < 2; ++q) e[q] *= is;
        }
        // e[] are the posteriors; sum_i w_i (l_i - log rho_i) for the per-row sum of w C
        float wcs = (e[0] > 0.f ? e[0] * (l[0] - lr2.x) : 0.f) +
                    (e[1] > 0.f ? e[1] * (l[1] - lr2.y) : 0.f);
        wcs = row16_sum(wcs);
        wcs += swz_xor16(wcs);
        {
            H hv[2], gv[2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                hv[q] = (H)e[q];
                gv[q] = (H)(e[q] - (float)hv[q]);
                accW[q] += e[q];
            }
            *(uint32_t *)(wsh + r * kKrWS + 4 * px) = __builtin_bit_cast(uint32_t, hv);
            *(uint32_t *)(wsh + BM * kKrWS + r * kKrWS + 4 * px) =
                __builtin_bit_cast(uint32_t, gv);
        }
        if (rv && px == 0) {
            acc_lse += (double)lse;
            acc_wc += (double)wcs;
            acc_rows += 1.0;
            if (A.flags & PF_STORE_LSE) A.lse[r0 + r] = (double)lse;
        }
        if constexpr (query) {
            // argmax (lowest column among equal maxima) and the gap to the runner-up
            float m1 = row16_max(fmaxf(e[0], e[1]));
            m1 = fmaxf(m1, swz_xor16(m1));
            int idx = 1 << 30;
#pragma unroll
            for (int q = 1; q >= 0; --q)
                if (cok[q] && e[q] == m1) idx = 2 * px + q;
#pragma unroll
            for (int o = 1; o < 32; o <<= 1) idx = min(idx, __shfl_xor(idx, o));
            float m2 = 0.f;
#pragma unroll
            for (int q = 0; q < 2; ++q)
                if (2 * px + q != idx) m2 = fmaxf(m2, e[q]);
            m2 = row16_max(m2);
            m2 = fmaxf(m2, swz_xor16(m2));
            if (rv) {
                const int64_t o = r0 + r - A.row_begin;
                if (A.post)
#pragma unroll
                    for (int q = 0; q < 2; ++q)
                        if (cok[q]) A.post[o * W + 2 * px + q] = e[q];
                if (px == 0) {
                    if (A.argmax) A.argmax[o] = idx;
                    if (A.margin) A.margin[o] = m1 - m2;
                }
            }
        }
        if (++nfw == kKrFlush) {                       // W_t sums: FP32 over 16 tiles
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                wacc[q] += (double)accW[q];
                accW[q] = 0.f;
            }
            nfw = 0;
        }
    };

    // ---- a5: U^T for this wave's frequencies, then the M-step on the wave's fragments of the
    // tile (rows Vs in LDS)
    auto mstep = [&](int rows, const float *rsv, const uint8_t *Vs) {
        f32x4 u4 = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const H8 bh = *(const H8 *)(wsh + rl * kKrWS + (32 * s + 8 * g) * 2);
            const H8 bl = *(const H8 *)(wsh + BM * kKrWS + rl * kKrWS + (32 * s + 8 * g) * 2);
            if constexpr (P == P_F16) {
                u4 = __builtin_amdgcn_mfma_f32_16x16x32_f16(el[s], bh, u4, 0, 0, 0);
                u4 = __builtin_amdgcn_mfma_f32_16x16x32_f16(eh[s], bl, u4, 0, 0, 0);
                u4 = __builtin_amdgcn_mfma_f32_16x16x32_f16(eh[s], bh, u4, 0, 0, 0);
            } else {
                u4 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(el[s], bh, u4, 0, 0, 0);
                u4 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(eh[s], bl, u4, 0, 0, 0);
                u4 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(eh[s], bh, u4, 0, 0, 0);
            }
        }
        // u4[q] = U[row rl][column 4 g + q] (before the row's storage scale)
        *(f32x4 *)(up + rl * kKrUS + 4 * g) = u4 * (rl < rows ? rsv[rl] : 0.f);
        asm volatile("" ::: "memory");           // a wave's LDS accesses complete in order
#pragma unroll
        for (int ks = 0; ks < KSS; ++ks) {
            const float2 U = *(const float2 *)(up + rl * kKrUS + um[ks]);
            const H8 v8 = *(const H8 *)(Vs + rl * LY.RS + (wave * KSS + ks) * 64 + g * 16);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float vr = (float)v8[2 * e], vi = (float)v8[2 * e + 1];
                sr[ks][e] = fmaf(U.x, vr, fmaf(-U.y, vi, sr[ks][e]));
                si[ks][e] = fmaf(U.x, vi, fmaf(U.y, vr, si[ks][e]));
            }
        }
        if (++nfl == kKrFlush) {
            fold();
            nfl = 0;
        }
    };

    // Software pipeline over this workgroup's tiles, two barriers per tile j: after the first
    // (tile j's partial correlations are in LDS) every wave forms its rows' posteriors of tile
    // j; after the second, it runs the products of tile j + 1, puts their partials in LDS, and
    // runs U and the M-step of tile j on its fragments of tile j, read again from LDS (a wave
    // whose products are done goes on to the M-step's vector work while the SIMD's other wave
    // still has products in the matrix core).  Tile t's rows sit in buffer t % 3 (copied during
    // tile t - 2, read by the products during tile t - 1 and by the M-step during tile t), its
    // row scales in slot t % 4.
    const int nm = (int)nmine;
    if (nm > 0) issue(0);
    if (nm > 1) issue(1);
    if (nm > 0) {                                // tile 0's products
        if (deep && nm > 1) {
            if (wave == 0) wait_vm<5>();
            else wait_vm<4>();
        } else {
            wait_vm<0>();
        }
        lds_barrier();
        products(0);
        put_red();
    }
    for (int j = 0, bc = 0; j < nm; ++j, bc = bc == kKrBufs - 1 ? 0 : bc + 1) {
        // tile j's partials are in LDS, and every wave is done with tile j - 1's rows and row
        // scales (whose buffer and slot tile j + 2 takes)
        lds_barrier();
        if (j + 2 < nm) issue(j + 2);
        const int64_t r0 = A.row_begin + (int64_t)blockIdx.x * BM + (int64_t)j * tstride;
        const int rows = (int)((A.row_end - r0) < BM ? (A.row_end - r0) : BM);
        const float *rsv = rsb + (j & 3) * 64;
        posteriors(r0, rows, rsv);
        // tile j + 1's copies have landed (tile j + 2's stay in flight) ...
        if (deep && j + 2 < nm) {
            if (wave == 0) wait_vm<5>();
            else wait_vm<4>();
        } else {
            wait_vm<0>();
        }
        // ... for every wave; every wave is done reading tile j's partials, and tile j's
        // posteriors are in LDS
        lds_barrier();
        if (j + 1 < nm) {
            products(bc == kKrBufs - 1 ? 0 : bc + 1);
            put_red();
        }
        if (accm) mstep(rows, rsv, smem + bc * BM * LY.RS);
    }
    fold();
#pragma unroll
    for (int q = 0; q < 2; ++q) wacc[q] += (double)accW[q];

    // ---- per-workgroup partials: S (2D), W_t (Wp), sum lse', sum w C, rows
    __syncthreads();
    const double *wsum = (const double *)(smem + LY.off_wacc);   // [16 row lanes][64 columns]
    if (A.partials) {
        double *Pp = A.partials + (int64_t)blockIdx.x * A.ncols;
        // value i of lane group g (i = 8 ks + 2 e + re/im) is real 2 d + (i & 1) of S, d = 16 (4
        // wave + ks) + 4 g + e
#pragma unroll
        for (int x = 0; x < 2; ++x) {
            const int i = rl + 16 * x, ks = i >> 3, e = (i >> 1) & 3;
            const int d = 16 * (wave * KSS + ks) + 4 * g + e;
            if (d < D) Pp[2 * d + (i & 1)] = accm ? s64[x] : 0.0;
        }
        if (tid < Wp) {
            double t = 0.0;
            for (int k = 0; k < 16; ++k) t += wsum[k * 64 + tid];
            Pp[2 * D + tid] = accm ? t : 0.0;
        }
        __syncthreads();
        put_pass_scalars(Pp + 2 * D + Wp, acc_lse, acc_wc, acc_rows, A.coef, (double *)smem);
    }
}

// ------------------------------------------------------------------------------------------
// Long-window FP32 correlation pass (full search over L rotations: the baseline the windowed
// forms are compared against), built as a matrix-core GEMM with the posterior and M-step as its
// epilogue.  A workgroup takes 128-row tiles; wave w owns the 16 rows 16 w .. 16 w + 15 and all
// Wp window columns of them (NTC 16-column tiles of accumulators).  The contraction over the 2D
// reals runs in 32-real chunks: each chunk's rows (16 KiB, 16-byte slots XOR-swizzled per row
// pair so that the fragment reads are conflict-free) and template rows (NTC x 2 KiB, in the
// template's fragment order) are copied global-to-LDS one chunk ahead into a double buffer.  The
// correlations are formed transposed (template fragments as the A operand, rows as B), so a lane
// ends with 4 NTC window columns of one row: the log-sum-exp and the posteriors need only its own
// registers and a reduction over the four lanes of the row.  Epilogue per tile:
//   * W_t: 16-lane DPP sums of the posteriors over the wave's rows, added over the waves in wave
//     order through LDS into one FP64 accumulator per column;
//   * U^T = E'^T w^T on matrix cores straight from the posterior registers (the contraction over
//     the window runs in the order the registers hold it; E' staged in LDS), left per wave in LDS;
//   * M-step on VALU: lane l takes entries 8 l .. 8 l + 7 (one frequency, Q % 8 == 0) of the
//     wave's 16 rows, re-read from global memory (on-die caches, mostly), FP64 sums per lane.
// Needs FP32 storage, D <= 512 with Q % 8 == 0, K <= 32 and Wp <= 384.

constexpr int kGmBM = 128;                // rows per tile (8 waves x 16)
constexpr int kGmKC = 32;                 // reals per contraction chunk
constexpr int kGmMaxNT = 24;              // window tiles (Wp <= 384)

struct GmLds {
    int stage, off_t, total_loop, off_e2, off_us, off_wt, off_sw, off_lr, total;
};
__host__ __device__ inline GmLds gm_lds(int NTC, int Wp, int K, int D) {
    GmLds l;
    const int vbytes = kGmBM * kGmKC * 4;                 // 16 KiB of rows per chunk
    l.off_t = vbytes;                                     // then NTC x 2 KiB of template
    l.stage = vbytes + NTC * 2 * 1024;
    l.total_loop = 2 * l.stage;
    // epilogue (the chunk buffers are idle then): E' (Wp x 2K floats), U^T blocks (8 waves x
    // 16 rows x 2K floats), the waves' column sums (8 x Wp floats)
    l.off_e2 = 0;
    l.off_us = align_up(((2 * K + 15) / 16) * NTC * 256 * 4, 16);
    l.off_wt = l.off_us + 8 * 16 * 2 * K * 4;
    int epi = l.off_wt + 8 * Wp * 4;
    // the waves' FP32 M-step sums (8 x 2D floats) go where E' was once it is consumed, unless
    // that area is too small (then after the column sums)
    const int swb = 8 * 2 * D * 4;
    l.off_sw = swb <= l.off_us ? 0 : align_up(epi, 16);
    if (l.off_sw) epi = l.off_sw + swb;
    l.off_lr = align_up(epi > l.total_loop ? epi : l.total_loop, 16);
    l.total = l.off_lr + Wp * 4 + 16;
    return l;
}

// s_waitcnt vmcnt(n) for a run-time n in [0, 15]
__device__ __forceinline__ void wait_vm_rt(int n) {
    switch (n) {
    case 0: wait_vm<0>(); break;
    case 1: wait_vm<1>(); break;
    case 2: wait_vm<2>(); break;
    case 3: wait_vm<3>(); break;
    case 4: wait_vm<4>(); break;
    case 5: wait_vm<5>(); break;
    case 6: wait_vm<6>(); break;
    case 7: wait_vm<7>(); break;
    case 8: wait_vm<8>(); break;
    case 9: wait_vm<9>(); break;
    default: wait_vm<0>(); break;
    }
}

template <int NTC, int QRY>
__global__ __launch_bounds__(kThreads) void pass_gm_kernel(PassArgs A) {
    static_assert(NTC >= 1 && NTC <= kGmMaxNT, "window tiles");
    constexpr bool query = QRY != 0;
    if ((A.flags & PF_CHECK_STOP) && *A.stopped) return;

    extern __shared__ __align__(16) uint8_t smem[];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int g = lane >> 4, j = lane & 15;
    const int D = A.D, K = A.K, W = A.W, Wp = A.Wp, K2 = 2 * A.K;
    const GmLds LY = gm_lds(NTC, Wp, K, D);
    float *lrs = (float *)(smem + LY.off_lr);
    for (int i = tid; i < Wp; i += kThreads) lrs[i] = A.logrho32[i];
    const float coef = (float)A.coef;
    const int NCH = A.Dp / kGmKC;                         // chunks per row
    const int KG = A.Dp / 16;                             // template k-groups per column tile
    // copies per wave per chunk: two 1 KiB row slices, and template slices w, w + 8, .. < 2 NTC
    const int ncopy = 2 + (2 * NTC + 7 - wave) / 8;
    const int64_t ntiles = (A.row_end - A.row_begin + kGmBM - 1) / kGmBM;

    // FP64 sums kept by thread t: M-step reals t and t + 512 (2D <= 1024), W_t column t
    double S64[2] = {0.0, 0.0};
    double Wacc = 0.0, acc_lse = 0.0, acc_wc = 0.0, acc_rows = 0.0;
    __syncthreads();

    // Full rounds of 128-row tiles over the grid, then the remaining rows split evenly over the
    // workgroups as one short tile each (a whole round of 128-row tiles for the remainder would
    // leave most workgroups idle while a few finish it); the waves of a short tile that hold no
    // rows skip their products.
    const int64_t nall = A.row_end - A.row_begin;
    const int64_t nfull = nall / ((int64_t)kGmBM * gridDim.x);
    const int64_t rem = nall - nfull * kGmBM * gridDim.x;
    (void)ntiles;
    for (int64_t tile = 0; tile < nfull + (rem > 0 ? 1 : 0); ++tile) {
        int64_t r0, rend;
        if (tile < nfull) {
            r0 = A.row_begin + (tile * gridDim.x + blockIdx.x) * kGmBM;
            rend = r0 + kGmBM;
        } else {
            const int64_t base = A.row_begin + nfull * kGmBM * gridDim.x;
            r0 = base + rem * blockIdx.x / gridDim.x;
            rend = base + rem * (blockIdx.x + 1) / gridDim.x;
        }
        if (rend <= r0) continue;                         // (no rows here: the whole workgroup)
        const bool wrows = r0 + 16 * wave < rend;         // this wave holds rows of the tile
        auto issue = [&](int c) {
            uint8_t *st = smem + (c & 1) * LY.stage;
            // rows: LDS slot p (16 B) of the chunk holds row p / 8, real slot (p % 8) ^ ((row >>
            // 1) & 7); wave w copies slots 64 (w + 8 x) .. + 63
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                const int p = 64 * (wave + 8 * x) + lane, r = p >> 3;
                const int sl = (p & 7) ^ ((r >> 1) & 7);
                const int64_t row = r0 + r < rend ? r0 + r : rend - 1;
                dma_to_lds<16>(A.V + row * A.rowbytes + (c * kGmKC + 4 * sl) * 4,
                               st + 64 * (wave + 8 * x) * 16);
            }
            // template: slice s = 2 nt + kk is k-group 2 c + kk of column tile nt (1 KiB)
            for (int s = wave; s < 2 * NTC; s += 8) {
                const int nt = s >> 1, kg = 2 * c + (s & 1);
                dma_to_lds<16>((const float *)A.Thi + (((int64_t)nt * KG + kg) * 64 + lane) * 4,
                               st + LY.off_t + s * 1024);
            }
        };
        // ---- a3: C^T for this wave's 16 rows over all window columns
        f32x4 acc[NTC];
#pragma unroll
        for (int t = 0; t < NTC; ++t) acc[t] = (f32x4){0.f, 0.f, 0.f, 0.f};
        issue(0);
        const int rr = 16 * wave + j;                     // this lane's row in the tile
        for (int c = 0; c < NCH; ++c) {
            wait_vm<0>();                                 // chunk c has landed (this wave's part)
            lds_barrier();                                // ... all of it; chunk c - 1 is consumed
            if (c + 1 < NCH) issue(c + 1);                // into the buffer chunk c - 1 used
            if (!wrows) continue;
            const uint8_t *st = smem + (c & 1) * LY.stage;
#pragma unroll
            for (int kk = 0; kk < 2; ++kk) {
                const int sl = (4 * kk + g) ^ ((rr >> 1) & 7);
                const float4 b = *(const float4 *)(st + rr * 128 + sl * 16);
#pragma unroll
                for (int t = 0; t < NTC; ++t) {
                    const float4 a = *(const float4 *)(st + LY.off_t + (2 * t + kk) * 1024 + lane * 16);
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, acc[t], 0, 0, 0);
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, acc[t], 0, 0, 0);
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b.z, acc[t], 0, 0, 0);
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b.w, acc[t], 0, 0, 0);
                }
            }
        }
        // acc[t][q] = C[row rr][column 16 t + 4 g + q]
        lds_barrier();                                    // the chunk buffers are free now
        // stage E' for the U product in the order its A operands are read: entry (mt, t, q, lane)
        // = E2[16 t + 4 (lane / 16) + q][16 mt + lane % 16] (zero past 2K)
        {
            float *e2s = (float *)(smem + LY.off_e2);
            const int MTs = (K2 + 15) / 16, n = MTs * NTC * 4 * 64;
            for (int x = tid; x < n; x += kThreads) {
                const int ln = x & 63, q = (x >> 6) & 3, t = (x >> 8) % NTC, mt = (x >> 8) / NTC;
                const int col = 16 * mt + (ln & 15), i = 16 * t + 4 * (ln >> 4) + q;
                e2s[x] = col < K2 ? A.E2[i * K2 + col] : 0.f;
            }
        }
        const int64_t row = r0 + rr;
        const bool rv = row < rend;

        // ---- a4: log-weights, log-sum-exp over the row's 4 lanes, posteriors (in acc)
        float mx = -INFINITY;
#pragma unroll
        for (int t = 0; t < NTC; ++t)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int col = 16 * t + 4 * g + q;
                const float l = (col < W && rv) ? acc[t][q] * coef + lrs[col] : -INFINITY;
                acc[t][q] = l;
                mx = fmaxf(mx, l);
            }
        mx = fmaxf(mx, swz_xor16(mx));
        mx = fmaxf(mx, __shfl_xor(mx, 32));
        float lse;
        if (A.flags & PF_LOAD_LSE) {
            lse = rv ? (float)A.lse[row] : 0.f;
        } else {
            float s = 0.f;
#pragma unroll
            for (int t = 0; t < NTC; ++t)
#pragma unroll
                for (int q = 0; q < 4; ++q) s += __expf(acc[t][q] - mx);   // exp(-inf) = 0
            s += swz_xor16(s);
            s += __shfl_xor(s, 32);
            lse = mx + __logf(s);
        }
        float wc = 0.f, m1 = 0.f;
#pragma unroll
        for (int t = 0; t < NTC; ++t)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int col = 16 * t + 4 * g + q;
                const float l = acc[t][q];
                const float w = rv ? __expf(l - lse) : 0.f;
                if (w > 0.f) wc += w * (l - lrs[col]);
                m1 = fmaxf(m1, w);
                acc[t][q] = w;
            }
        wc += swz_xor16(wc);
        wc += __shfl_xor(wc, 32);
        if (rv && g == 0) {
            acc_lse += (double)lse;
            acc_wc += (double)wc;
            acc_rows += 1.0;
            if (A.flags & PF_STORE_LSE) A.lse[row] = (double)lse;
        }
        if constexpr (query) {
            // argmax (lowest column among equal maxima) and the gap to the runner-up
            m1 = fmaxf(m1, swz_xor16(m1));
            m1 = fmaxf(m1, __shfl_xor(m1, 32));
            int idx = 1 << 30;
#pragma unroll
            for (int t = NTC - 1; t >= 0; --t)
#pragma unroll
                for (int q = 3; q >= 0; --q)
                    if (acc[t][q] == m1 && 16 * t + 4 * g + q < W) idx = 16 * t + 4 * g + q;
            idx = min(idx, __shfl_xor(idx, 16));
            idx = min(idx, __shfl_xor(idx, 32));
            float m2 = 0.f;
#pragma unroll
            for (int t = 0; t < NTC; ++t)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (16 * t + 4 * g + q != idx) m2 = fmaxf(m2, acc[t][q]);
            m2 = fmaxf(m2, swz_xor16(m2));
            m2 = fmaxf(m2, __shfl_xor(m2, 32));
            if (rv) {
                const int64_t o = row - A.row_begin;
                if (A.post) {
#pragma unroll
                    for (int t = 0; t < NTC; ++t)
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            if (16 * t + 4 * g + q < W) A.post[o * W + 16 * t + 4 * g + q] = acc[t][q];
                }
                if (g == 0) {
                    if (A.argmax) A.argmax[o] = idx;
                    if (A.margin) A.margin[o] = m1 - m2;
                }
            }
        }
        if (!(A.flags & PF_ACC_M)) {
            __syncthreads();                              // before the next tile's copies
            continue;
        }

        // ---- W_t: column sums over the wave's 16 rows (DPP), then over the waves in order
        float *wt = (float *)(smem + LY.off_wt);
#pragma unroll
        for (int t = 0; t < NTC; ++t)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float s = row16_sum(acc[t][q]);
                if (((4 * t + q) & 15) == j) wt[wave * Wp + 16 * t + 4 * g + q] = s;
            }
        // ---- a5: U^T = E'^T w^T, contraction over the window in register order: k-step (t, q)
        // pairs lane group g with window column 16 t + 4 g + q
        const float *e2s = (const float *)(smem + LY.off_e2);
        float *us = (float *)(smem + LY.off_us) + wave * 16 * K2;
        lds_barrier();                                    // E' staged, column sums written
        if (tid < Wp) {
            float s = 0.f;
            for (int w2 = 0; w2 < 8; ++w2) s += wt[w2 * Wp + tid];
            Wacc += (double)s;
        }
        const int MT = (K2 + 15) / 16;
        for (int mt = 0; mt < MT; ++mt) {
            const float *ep = e2s + mt * NTC * 256 + lane;
            f32x4 u4 = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int t = 0; t < NTC; ++t)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    u4 = __builtin_amdgcn_mfma_f32_16x16x4f32(ep[(4 * t + q) * 64], acc[t][q], u4,
                                                              0, 0, 0);
            // u4[q] = U[row j][16 mt + 4 g + q]
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (16 * mt + 4 * g + q < K2) us[j * K2 + 16 * mt + 4 * g + q] = u4[q];
        }
        asm volatile("" ::: "memory");                    // a wave's LDS accesses complete in order
        // M-step: entries d = 8 lane + e of the wave's 16 rows (FP32 over the 16 rows), then the
        // waves' sums added in wave order into the FP64 sums (E' staging area reused)
        float *swv = (float *)(smem + LY.off_sw);         // 8 waves x 2D floats
        lds_barrier();                                    // every wave is done reading E'
        if (8 * lane < D) {                               // (waves without rows write zeros)
            const int k = (8 * lane) / A.Q;
            float sr[8], si[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) sr[e] = si[e] = 0.f;
#pragma unroll 4
            for (int jr = 0; jr < (wrows ? 16 : 0); ++jr) {
                const int64_t rw = r0 + 16 * wave + jr;
                const int64_t rc = rw < rend ? rw : rend - 1;
                const float4 *src = (const float4 *)(A.V + rc * A.rowbytes) + 4 * lane;
                float4 v[4];
#pragma unroll
                for (int x = 0; x < 4; ++x) v[x] = src[x];
                const float ur = us[jr * K2 + k], ui = us[jr * K2 + K + k];   // 0 past the end
#pragma unroll
                for (int x = 0; x < 4; ++x) {
                    sr[2 * x] += ur * v[x].x - ui * v[x].y;
                    si[2 * x] += ur * v[x].y + ui * v[x].x;
                    sr[2 * x + 1] += ur * v[x].z - ui * v[x].w;
                    si[2 * x + 1] += ur * v[x].w + ui * v[x].z;
                }
            }
            float *o = swv + wave * 2 * D + 16 * lane;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                o[2 * e] = sr[e];
                o[2 * e + 1] = si[e];
            }
        }
        lds_barrier();
#pragma unroll
        for (int x = 0; x < 2; ++x) {
            const int r = tid + x * kThreads;
            if (r < 2 * D) {
                float s8 = 0.f;
                for (int w2 = 0; w2 < 8; ++w2) s8 += swv[w2 * 2 * D + r];
                S64[x] += (double)s8;
            }
        }
        __syncthreads();                                  // LDS reused by the next tile's copies
    }

    // ---- per-workgroup partials: S (the waves' sums in wave order), W_t, sum lse', sum w C, rows
    if (A.partials) {
        double *Pp = A.partials + (int64_t)blockIdx.x * A.ncols;
        const bool accm = (A.flags & PF_ACC_M) != 0;
#pragma unroll
        for (int x = 0; x < 2; ++x) {
            const int r = tid + x * kThreads;
            if (r < 2 * D) Pp[r] = accm ? S64[x] : 0.0;
        }
        if (tid < Wp) Pp[2 * D + tid] = accm ? Wacc : 0.0;
        __syncthreads();
        put_pass_scalars(Pp + 2 * D + Wp, acc_lse, acc_wc, acc_rows, A.coef, (double *)smem);
    }
}

// ------------------------------------------------------------------------------------------
// Factored E(+M) pass: the correlations through per-frequency sums, an exact rewrite of the
// contraction (a rotation is one phase per angular frequency, §I eq. (3)):
//   Re <v_j, R_{o_i} a> = Re sum_k c_jk exp(-i k theta_i),   c_jk = sum_q conj(v_jkq) a_kq.
// Per row this costs 4D + 4KW flops instead of 4DW, no template exists, and the pass is a stream
// over the rows.  Each wave owns fac_rpw rows of a tile of 8 fac_rpw rows and holds them in
// registers (lane l: entries EPL l .. EPL l + EPL - 1, so D = 64 EPL with EPL = 8 for D = 512;
// Q/EPL lanes share an angular frequency), while the next tile's rows load (waves 0-3 issue their
// loads at the top of a tile, waves 4-7 after the first barrier, so that the two halves' loads do
// not queue behind each other).  For D = 2048 in one 16-bit plane (EPL = 16) a row is split over
// a pair of waves: wave w holds half h = w % 2 of the rows of its row group w / 2 (virtual lane
// 64 h + lane: entries 16 (64 h + lane) ..).  c (FMA chains, then a branch-free DPP sum over the
// lanes of a frequency; scaled by the row factor coef s_j) goes to LDS;
// C = [Re c | Im c] . [cos; sin] and U = w [Re E | Im E] are FP32 matrix-core products against
// the phase table (fragments in registers when Wp <= 64, with a permuted k order so that the A
// operands are 16-byte LDS words; otherwise from the LDS grid phase table or from L2); the
// posteriors as in the other passes (tile_rows_short for Wp <= 64 without queries); the M-step
// from the rows in registers, the eight waves' partial sums added in wave order into per-entry
// FP64 accumulators (EPL = 8: the waves' FP32 partials summed by entry owners; EPL = 16: the row
// groups add theirs in order into an FP64 copy of S in LDS).

// rows per wave per tile: 2 for the 16-word row formats (FP32, bf16x3), 4 for one 16-bit plane
__host__ __device__ constexpr int fac_rpw(int prec, int epl = 8) {
    return (epl == 8 && (prec == P_F32 || prec == P_BF16X3)) ? 2 : 4;
}
// rows per tile: 8 waves (EPL = 8) or 4 pairs of waves (EPL = 16) times the rows per wave
__host__ __device__ constexpr int fac_bm(int prec, int epl = 8) {
    return (epl == 16 ? 4 : 8) * fac_rpw(prec, epl);
}
constexpr int kFacFlush = 16;                 // tiles summed in FP32 before the FP64 flush
constexpr int kFacFlush16 = 8;                // ... with 16 entries per lane

constexpr int kFacPhLds = 2048;               // grid phase table staged in LDS up to this L

struct FacLds {
    int CBW, CSW, off_cs, off_u, off_sw, off_f, off_lr, off_a, off_ph, off_wb, total;
};
// PHL: entries of the grid phase table kept in LDS (0: none); WBF: bf16 hi + lo planes of the
// posteriors (256 B per row) for the bf16 matrix-core U product
__host__ __device__ inline FacLds fac_lds(int K, int D, int Wp, int KCM, int BM, int EPL = 8,
                                          int PHL = 0, bool WBF = false) {
    FacLds l;
    l.CBW = 4 * KCM + 4;                       // [Re c | Im c | 0 ..], conflict-free A reads
    l.CSW = (Wp > 64 ? Wp : 64) + 4;           // columns past Wp stay zero (register U path)
    l.off_cs = align_up(BM * l.CBW * 4, 16);
    l.off_u = align_up(l.off_cs + BM * l.CSW * 4, 16);
    l.off_sw = align_up(l.off_u + BM * K * 8, 16);
    l.off_f = align_up(l.off_sw + (EPL == 16 ? D * 16 : 8 * (9 * D / 8) * 8), 16);
    l.off_lr = l.off_f + 2 * BM * 4;
    l.off_a = align_up(l.off_lr + Wp * 4, 16);
    l.off_ph = align_up(l.off_a + D * 8, 16);
    l.off_wb = align_up(l.off_ph + PHL * 8, 16);
    l.total = l.off_wb + (WBF ? BM * 256 : 0);
    return l;
}

// The factored pass's C and U products with the phase factors read from the grid phase table in
// LDS (ph[m] = (cos, sin)(2 pi m / L), E[i, k] = ph[(k (lo + i)) mod L]) instead of the E2 table
// in L2.  C: wave w takes the column tiles w, w + 8, .. of the BM x Wp tile.
template <int BM, int KCM>
__device__ __forceinline__ void fac_c_ph(const float *cb, int CBW, const float2 *ph, int L, int lo,
                                         int W, int NT, int K,
                                         const float *lrs, float *Cs, int CSW) {
    constexpr int MT = BM / 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, c = lane & 15;
    for (int p = wave; p < MT * NT; p += 8) {
        const int m = p % MT, n = p / MT;
        const int i = 16 * n + c;
        const int mo = i < W ? (lo + i) % L : 0;
        f32x4 cacc = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll 8
        for (int kk = 0; kk < KCM; ++kk) {
            const int colk = 4 * kk + g;
            float b = 0.f;
            if (i < W && colk < 2 * K) {
                const int kq = colk < K ? colk : colk - K;
                const float2 e = ph[(kq * mo) % L];
                b = colk < K ? e.x : e.y;
            }
            const float a = cb[(16 * m + c) * CBW + colk];
            cacc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, cacc, 0, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = 16 * m + 4 * g + q;
            Cs[row * CSW + i] = cacc[q] + lrs[i];
        }
    }
}

// U (BM x 2K) = w (BM x Wp) . [Re E | Im E] with E from the LDS grid phase table; wave w takes
// the 16-column tiles w, w + 8, .. of U; lane (g, rl) steps its window index i = 4 kk + g, so
// its phase index moves by 4 k (mod L) per step.
template <int BM>
__device__ __forceinline__ void u_mfma_ph(const float *Cs, int CSW, const float2 *ph, int L,
                                          int lo, int W, int Wp, int K, const float *rowu,
                                          float2 *Us) {
    constexpr int MS = BM / 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, rl = lane & 15;
    const int NTU = (2 * K + 15) / 16, KG = Wp / 4;
    for (int nt = wave; nt < NTU; nt += kThreads / 64) {
        f32x4 acc[MS];
#pragma unroll
        for (int m = 0; m < MS; ++m) acc[m] = (f32x4){0.f, 0.f, 0.f, 0.f};
        const int col = nt * 16 + rl;
        const bool cok = col < 2 * K;
        const int kq = col < K ? col : col - K;
        const bool im = col >= K;
        int mi = cok ? (int)(((int64_t)kq * ((lo + g) % L)) % L) : 0;
        const int step = cok ? (4 * kq) % L : 0;
#pragma unroll 4
        for (int kk = 0; kk < KG; ++kk) {
            const int i = 4 * kk + g;
            float b = 0.f;
            if (cok && i < W) {
                const float2 e = ph[mi];
                b = im ? e.y : e.x;
            }
            mi += step;
            if (mi >= L) mi -= L;
#pragma unroll
            for (int m = 0; m < MS; ++m) {
                const float a = Cs[(m * 16 + rl) * CSW + kk * 4 + g];
                acc[m] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[m], 0, 0, 0);
            }
        }
        if (cok) {
#pragma unroll
            for (int m = 0; m < MS; ++m)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int row = m * 16 + 4 * g + q;
                    const float v = acc[m][q] * rowu[row];
                    if (col < K)
                        Us[row * K + col].x = v;
                    else
                        Us[row * K + col - K].y = v;
                }
        }
    }
}

// U (BM x 2K) = w (BM x 64) . [Re E | Im E] for windows of at most 64 offsets, this wave's B
// fragments in registers, scaled by rowu (or without the row scale, which the M-step then
// applies, when rowu is null).  The sum over the window
// runs in a permuted order: lane (g, rl) takes window index 16 g + kk at k-step kk
// (ereg[kk] = E2[16 g + kk][ucol]), so its A values are 16 consecutive posteriors of row rl, read
// as four 16-byte words; with one row tile, even and odd k-steps accumulate in two chains.
template <int BM>
__device__ __forceinline__ void u_fac_reg(const float *Cs, int CSW, const float (&ereg)[16],
                                          int K, const float *rowu, float2 *Us, int ucol) {
    constexpr int MS = BM / 16;
    const int lane = threadIdx.x & 63, g = lane >> 4, rl = lane & 15;
    if ((ucol & ~15) >= 2 * K) return;             // this wave's U column tile is past 2K
    constexpr int NCH = MS == 1 ? 2 : 1;           // accumulator chains per row tile
    f32x4 acc[MS][NCH];
#pragma unroll
    for (int m = 0; m < MS; ++m)
#pragma unroll
        for (int h = 0; h < NCH; ++h) acc[m][h] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int m = 0; m < MS; ++m) {
        const float4 *ar = (const float4 *)(Cs + (m * 16 + rl) * CSW + 16 * g);
        float4 a4[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) a4[t] = ar[t];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            constexpr int o = NCH - 1;
            acc[m][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4[t].x, ereg[4 * t], acc[m][0], 0, 0, 0);
            acc[m][o] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4[t].y, ereg[4 * t + 1], acc[m][o], 0, 0, 0);
            acc[m][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4[t].z, ereg[4 * t + 2], acc[m][0], 0, 0, 0);
            acc[m][o] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4[t].w, ereg[4 * t + 3], acc[m][o], 0, 0, 0);
        }
    }
    if (ucol < 2 * K) {
#pragma unroll
        for (int m = 0; m < MS; ++m)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = m * 16 + 4 * g + q;
                float v = NCH == 2 ? acc[m][0][q] + acc[m][NCH - 1][q] : acc[m][0][q];
                if (rowu) v *= rowu[row];
                if (ucol < K)
                    Us[row * K + ucol].x = v;
                else
                    Us[row * K + ucol - K].y = v;
            }
    }
}

// The same U product in bf16 hi + lo on matrix cores (three 16x16x32 products per k-step, FP32
// accumulation, the lo x lo term left out): A from the bf16 planes of the posteriors (row rl,
// window indices 32 s + 8 g .. + 7), B = hi / lo of E2[32 s + 8 g + t][ucol], t = 0 .. 7.
__device__ __forceinline__ void u_fac_bf(const uint8_t *wb, const bf16x8 (&bh)[2],
                                         const bf16x8 (&bl)[2], int K, float2 *Us, int ucol) {
    const int lane = threadIdx.x & 63, g = lane >> 4, rl = lane & 15;
    if ((ucol & ~15) >= 2 * K) return;             // this wave's U column tile is past 2K
    f32x4 acc0 = (f32x4){0.f, 0.f, 0.f, 0.f}, acc1 = acc0;
    const uint8_t *ar = wb + rl * 256 + 16 * g;
#pragma unroll
    for (int st = 0; st < 2; ++st) {
        const bf16x8 AH = *(const bf16x8 *)(ar + 64 * st);
        const bf16x8 AL = *(const bf16x8 *)(ar + 128 + 64 * st);
        acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(AH, bh[st], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(AL, bh[st], acc1, 0, 0, 0);
        acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(AH, bl[st], acc0, 0, 0, 0);
    }
    if (ucol < 2 * K) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = 4 * g + q;
            const float v = acc0[q] + acc1[q];
            if (ucol < K)
                Us[row * K + ucol].x = v;
            else
                Us[row * K + ucol - K].y = v;
        }
    }
}

// hi and lo bf16x8 of eight FP32 values
__device__ __forceinline__ void split_bf16x8(const float (&x)[8], bf16x8 &h, bf16x8 &l) {
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        h[t] = (__bf16)x[t];
        l[t] = (__bf16)(x[t] - (float)h[t]);
    }
}

// Words of one stored row for lane l (entries EPL l .. EPL l + EPL - 1): FP32 2 EPL words
// (re, im per entry); bf16x3 EPL hi words then EPL lo words; fp16 / bf16 EPL words.
template <int P, int EPL = 8>
struct FacRow {
    static constexpr int WPL = (P == P_F32 || P == P_BF16X3) ? 2 * EPL : EPL;
    u32x4 w[WPL / 4];
    __device__ __forceinline__ void load(const uint8_t *row, int Dp, int lane) {
        if constexpr (P == P_F32) {
            const u32x4 *p = (const u32x4 *)(row + 8 * EPL * lane);
#pragma unroll
            for (int t = 0; t < WPL / 4; ++t) w[t] = p[t];
        } else {
            const u32x4 *p = (const u32x4 *)(row + 4 * EPL * lane);
#pragma unroll
            for (int t = 0; t < EPL / 4; ++t) w[t] = p[t];
            if constexpr (P == P_BF16X3) {
                const u32x4 *q = (const u32x4 *)(row + 2 * Dp + 4 * EPL * lane);
#pragma unroll
                for (int t = 0; t < EPL / 4; ++t) w[EPL / 4 + t] = q[t];
            }
        }
    }
    __device__ __forceinline__ float2 entry(int e) const {
        if constexpr (P == P_F32) {
            return make_float2(__uint_as_float(w[e >> 1][(e & 1) * 2]),
                               __uint_as_float(w[e >> 1][(e & 1) * 2 + 1]));
        } else if constexpr (P == P_F16) {
            const uint32_t x = w[e >> 2][e & 3];
            const _Float16 *h = (const _Float16 *)&x;
            return make_float2((float)h[0], (float)h[1]);
        } else {
            const uint32_t x = w[e >> 2][e & 3];
            float re = __uint_as_float(x << 16), im = __uint_as_float(x & 0xffff0000u);
            if constexpr (P == P_BF16X3) {
                const uint32_t y = w[EPL / 4 + (e >> 2)][e & 3];
                re += __uint_as_float(y << 16);
                im += __uint_as_float(y & 0xffff0000u);
            }
            return make_float2(re, im);
        }
    }
};

// WIDE = 0: Wp <= 64 (phase fragments in registers); 1: longer windows.  KCM = k-steps of 4
// columns over [Re c | Im c] (2K <= 4 KCM).  EPL = entries per lane (D = 64 EPL).
template <int P, int WIDE, int KCM, int EPL>
__global__ __launch_bounds__(kThreads) void pass_fac_kernel(PassArgs A) {
    static_assert(P != P_F64, "matrix-core precisions");
    static_assert(EPL == 8 || (EPL == 16 && WIDE && (P == P_F16 || P == P_BF16)),
                  "16 entries per lane: one 16-bit plane, phase factors not in registers");
    constexpr bool HR = EPL == 16;                 // a row over a pair of waves
    constexpr int NVL = HR ? 128 : 64;             // virtual lanes of a row: D = NVL EPL
    constexpr int RPW = fac_rpw(P, EPL), BM = fac_bm(P, EPL), DPT = NVL * EPL / kThreads;
    // bf16x3 storage, windows up to 64, 2K up to 64: the C and U products in bf16 hi + lo on
    // matrix cores (c and the posteriors kept as bf16 hi + lo planes in LDS)
    constexpr bool BFX = P == P_BF16X3 && !WIDE && KCM == 16;
    static_assert(!BFX || BM == 16, "one 16-row tile");
    if ((A.flags & PF_CHECK_STOP) && *A.stopped) return;

    extern __shared__ __align__(16) uint8_t smem[];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int g = lane >> 4, c = lane & 15;
    const int K = A.K, D = A.D, Wp = A.Wp, NT = Wp / 16;
    const int hh = HR ? (wave & 1) : 0, rg = HR ? (wave >> 1) : wave;   // half, row group
    const int vl = 64 * hh + lane;                 // this lane's place in the row
    // long windows on the grid: the phase factors come from an LDS copy of the grid phase table
    const bool use_ph = WIDE && A.grid && A.L <= kFacPhLds;
    const FacLds LY = fac_lds(K, D, Wp, KCM, BM, EPL, use_ph ? A.L : 0, BFX);
    uint8_t *wb = smem + LY.off_wb;                // (BFX) bf16 planes of the posteriors
    float2 *phs = (float2 *)(smem + LY.off_ph);
    if (use_ph)
        for (int m = tid; m < A.L; m += kThreads)
            phs[m] = make_float2((float)A.phase[m].x, (float)A.phase[m].y);
    float *cb = (float *)smem;
    float *Cs = (float *)(smem + LY.off_cs);
    float2 *Us = (float2 *)(smem + LY.off_u);
    float2 *Sw = (float2 *)(smem + LY.off_sw);
    float *rowu = (float *)(smem + LY.off_f) + BM;    // the row scales s_j
    const float coef = (float)A.coef;
    float *lrs = (float *)(smem + LY.off_lr);
    // a (FP32) stored lane-major: entry e of lane l at [e][l], so the lanes' reads are
    // conflict-free
    float2 *as = (float2 *)(smem + LY.off_a);
    for (int i = tid; i < Wp; i += kThreads) lrs[i] = A.logrho32[i];
    for (int d = tid; d < D; d += kThreads)
        as[(d % EPL) * NVL + d / EPL] = make_float2((float)A.a[2 * d], (float)A.a[2 * d + 1]);
    if constexpr (HR)
        for (int d = tid; d < D; d += kThreads) ((double2 *)Sw)[d] = make_double2(0.0, 0.0);

    // this lane's entries and their coefficients a (FP32), its angular frequency and lane group
    const int d0 = EPL * vl;
    const int LPK = A.Q / EPL;
    const int kl = d0 / A.Q;
    float lpk_f[4];                                // the DPP steps of the LPK-lane sums
#pragma unroll
    for (int t = 0; t < 4; ++t) lpk_f[t] = LPK > (1 << t) ? 1.f : 0.f;
    // columns 2K .. 4 KCM - 1 of the c rows stay zero for the whole pass (BFX: the c rows are a
    // bf16 hi plane of 64 entries followed by a lo plane, zero past 2K in both)
    if constexpr (BFX) {
        for (int x = tid; x < BM * LY.CBW; x += kThreads) cb[x] = 0.f;
    } else {
        for (int x = tid; x < BM * (4 * KCM - 2 * K); x += kThreads) {
            const int j = x / (4 * KCM - 2 * K);
            cb[j * LY.CBW + 2 * K + x % (4 * KCM - 2 * K)] = 0.f;
        }
    }
    __syncthreads();
    // two-row formats, short windows: values that stay fixed for the pass held in registers (the
    // lane's coefficients, its C-epilogue log-prior, its four posterior-step log-priors)
    constexpr bool kHold = !HR && !WIDE && RPW == 2;
    float2 ahold[kHold ? EPL : 1];
    float4 lrhold = make_float4(0.f, 0.f, 0.f, 0.f);
    float lrc = 0.f;
    if constexpr (kHold) {
#pragma unroll
        for (int e = 0; e < EPL; ++e) ahold[e] = as[e * NVL + vl];
        if (tid < 16 * BM) lrhold = *(const float4 *)(lrs + 4 * (tid & 15));
        if ((wave & 3) < NT) lrc = lrs[16 * (wave & 3) + c];
    }
    // C product: wave w computes rows 16 (w >> 2) .. of window tile (w & 3) (Wp <= 64); the sum
    // over [Re c | Im c] runs in a permuted order (lane group g takes columns KCM g .. KCM g +
    // KCM - 1, read as 16-byte words), so its B fragments are E2[16 n + c][KCM g + kk] (zero past
    // 2K)
    float cfr[BFX ? 1 : KCM];
    const int cm = wave >> 2, cn = wave & 3;       // (16-row tiles: waves 0-3 only)
    if constexpr (!WIDE && !BFX) {
#pragma unroll
        for (int kk = 0; kk < KCM; ++kk) {
            const int col = KCM * g + kk, i = 16 * cn + c;
            cfr[kk] = (col < 2 * K && i < Wp) ? A.E2[(int64_t)i * 2 * K + col] : 0.f;
        }
    }
    // BFX: B fragments of C (k-step s: E2[16 cn + c][32 s + 8 g + t]) and of U
    // (E2[32 s + 8 g + t][ucol]), hi and lo
    bf16x8 cbh[BFX ? 2 : 1], cbl[BFX ? 2 : 1], ubh[BFX ? 2 : 1], ubl[BFX ? 2 : 1];
    // U product: wave w computes U columns 16 (w ^ 4) + c over 16 k-steps (Wp <= 64): for
    // 2K <= 64 the upper four waves, while wave 0 takes the W column sums; window index
    // 16 g + kk at k-step kk (u_fac_reg)
    const int ucol = (wave ^ 4) * 16 + c;
    float ereg[BFX ? 1 : 16];
    if constexpr (!WIDE && !BFX) {
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            const int i = 16 * g + kk;
            ereg[kk] = (i < Wp && ucol < 2 * K) ? A.E2[(int64_t)i * 2 * K + ucol] : 0.f;
        }
    }
    if constexpr (BFX) {
#pragma unroll
        for (int st = 0; st < 2; ++st) {
            float xc[8], xu[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int kc = 32 * st + 8 * g + t, ic = 16 * cn + c;
                xc[t] = (kc < 2 * K && ic < Wp) ? A.E2[(int64_t)ic * 2 * K + kc] : 0.f;
                const int iu = 32 * st + 8 * g + t;
                xu[t] = (iu < Wp && ucol < 2 * K) ? A.E2[(int64_t)iu * 2 * K + ucol] : 0.f;
            }
            split_bf16x8(xc, cbh[st], cbl[st]);
            split_bf16x8(xu, ubh[st], ubl[st]);
        }
    }

    PassAcc<DPT> acc;
    acc.init();
    const int64_t ntiles = (A.row_end - A.row_begin + BM - 1) / BM;
    FacRow<P, EPL> vn[RPW];
    float rsn[RPW];
    auto load_tile = [&](int64_t t) {
        const int64_t rb = A.row_begin + t * BM + RPW * rg;
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            const int64_t row = rb + r < A.row_end ? rb + r : A.row_end - 1;
            // (the second half of a split row starts after D/2 entries of 4 bytes)
            vn[r].load(A.V + row * A.rowbytes + (HR ? hh * (D / 2) * 4 : 0), A.Dp, lane);
            rsn[r] = A.rowscale ? A.rowscale[row] : 1.0f;
        }
    };
    float sr[EPL], si[EPL];                   // this lane's M-step partials (FP32)
#pragma unroll
    for (int e = 0; e < EPL; ++e) sr[e] = si[e] = 0.f;
    int nacc = 0;
    auto flush = [&]() {
      if constexpr (HR) {
        // the four row groups add their FP32 partials into the FP64 copy of S in order (the two
        // halves of a group own disjoint entries)
        double2 *Sd = (double2 *)Sw;
        for (int w = 0; w < 4; ++w) {
            if (rg == w)
#pragma unroll
                for (int e = 0; e < EPL; ++e) {
                    double2 t = Sd[d0 + e];
                    t.x += (double)sr[e];
                    t.y += (double)si[e];
                    Sd[d0 + e] = t;
                }
            lds_barrier();
        }
      } else {
        // wave w's partials at [w][9 (d / 8) + d % 8] (padded: the lanes' writes spread over
        // the banks)
        const int SWS = 9 * D / 8;
#pragma unroll
        for (int e = 0; e < EPL; ++e) Sw[wave * SWS + 9 * lane + e] = make_float2(sr[e], si[e]);
        lds_barrier();
#pragma unroll
        for (int cc = 0; cc < DPT; ++cc) {
            const int d = tid + cc * kThreads;
            if (d < D) {
                const int o = 9 * (d >> 3) + (d & 7);
                float2 s = Sw[o];
#pragma unroll
                for (int w = 1; w < 8; ++w) {
                    const float2 t = Sw[w * SWS + o];
                    s.x += t.x;
                    s.y += t.y;
                }
                acc.S[cc].x += (double)s.x;
                acc.S[cc].y += (double)s.y;
            }
        }
      }
#pragma unroll
        for (int e = 0; e < EPL; ++e) sr[e] = si[e] = 0.f;
        nacc = 0;
    };
    int64_t tile = blockIdx.x;
    // EPL = 8: the next tile's rows load into registers while this one is used; EPL = 16 loads
    // each tile at its start (the register file holds one tile of its rows)
    constexpr bool kPrefetch = !HR;
    if (kPrefetch && tile < ntiles) load_tile(tile);
    for (; tile < ntiles; tile += gridDim.x) {
        const int64_t r0 = A.row_begin + tile * BM;
        const int rows = (int)((A.row_end - r0) < BM ? (A.row_end - r0) : BM);
        if constexpr (!kPrefetch) load_tile(tile);
        FacRow<P, EPL> vc[RPW];
        float rsc[RPW];
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            vc[r] = vn[r];
            rsc[r] = rsn[r];
        }
        // the next tile's rows: waves 0-3 issue their loads now, waves 4-7 after the c barrier
        // (issued all at once, the later waves' loads queue behind the earlier ones')
        const bool pf = kPrefetch && tile + gridDim.x < ntiles;
        if (pf && wave < 4) load_tile(tile + gridDim.x);

        // ---- c_jk for this wave's rows; row factors.  EPL = 8: the lane's coefficients are read
        // from LDS once per tile, ahead of the rows
        float2 areg[HR ? 1 : EPL];
        if constexpr (kHold) {
#pragma unroll
            for (int e = 0; e < EPL; ++e) areg[e] = ahold[e];
        } else if constexpr (!HR) {
#pragma unroll
            for (int e = 0; e < EPL; ++e) areg[e] = as[e * NVL + vl];
        }
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            const int j = RPW * rg + r;
            float cr = 0.f, ci = 0.f;
#pragma unroll
            for (int e = 0; e < EPL; ++e) {
                const float2 v = vc[r].entry(e);
                float2 av;
                if constexpr (HR) av = as[e * NVL + vl]; else av = areg[e];
                cr = fmaf(v.x, av.x, cr);                 // Re conj(v) a
                cr = fmaf(v.y, av.y, cr);
                ci = fmaf(v.x, av.y, ci);                 // Im conj(v) a
                ci = fmaf(-v.y, av.x, ci);
            }
            cr = lanes_sum_dpp(cr, lpk_f);
            ci = lanes_sum_dpp(ci, lpk_f);
            for (int o = 16; o < LPK; o <<= 1) {
                cr += __shfl_xor(cr, o);
                ci += __shfl_xor(ci, o);
            }
            // c scaled by the row factor coef s_j: the C products then need no epilogue scaling
            const float u = j < rows ? rsc[r] : 1.0f;
            if ((lane & (LPK - 1)) == 0) {
                const float xr = cr * (coef * u), xi = ci * (coef * u);
                if constexpr (BFX) {
                    __bf16 *ch = (__bf16 *)(cb + j * LY.CBW);     // hi [0, 64), lo [64, 128)
                    const __bf16 hr = (__bf16)xr, hi_ = (__bf16)xi;
                    ch[kl] = hr;
                    ch[K + kl] = hi_;
                    ch[64 + kl] = (__bf16)(xr - (float)hr);
                    ch[64 + K + kl] = (__bf16)(xi - (float)hi_);
                } else {
                    cb[j * LY.CBW + kl] = xr;
                    cb[j * LY.CBW + K + kl] = xi;
                }
            }
            if (lane == 0) rowu[j] = u;
        }
        lds_barrier();
        if (pf && wave >= 4) load_tile(tile + gridDim.x);

        // ---- C = [Re c | Im c] . E2^T on FP32 matrix cores -> l' = coef C / s_j + log rho
        if constexpr (BFX) {
          if (wave < 4) {
            f32x4 cacc = (f32x4){0.f, 0.f, 0.f, 0.f}, cacc1 = cacc;
            const uint8_t *arow = (const uint8_t *)(cb + c * LY.CBW) + 16 * g;
#pragma unroll
            for (int st = 0; st < 2; ++st) {
                const bf16x8 AH = *(const bf16x8 *)(arow + 64 * st);
                const bf16x8 AL = *(const bf16x8 *)(arow + 128 + 64 * st);
                cacc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(AH, cbh[st], cacc, 0, 0, 0);
                cacc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(AL, cbh[st], cacc1, 0, 0, 0);
                cacc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(AH, cbl[st], cacc, 0, 0, 0);
            }
            const int col = 16 * cn + c;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = 4 * g + q;
                Cs[row * LY.CSW + col] = cn < NT ? cacc[q] + cacc1[q] + (kHold ? lrc : lrs[col]) : 0.f;
            }
          }
        } else if constexpr (!WIDE) {
          if (16 * cm < BM) {
            // even / odd k-steps in two chains (one for KCM = 32, which has no registers to spare)
            f32x4 cacc = (f32x4){0.f, 0.f, 0.f, 0.f}, cacc1 = cacc;
            const float4 *arow = (const float4 *)(cb + (16 * cm + c) * LY.CBW + KCM * g);
            float4 a4[KCM / 4];
#pragma unroll
            for (int t = 0; t < KCM / 4; ++t) a4[t] = arow[t];
#pragma unroll
            for (int t = 0; t < KCM / 4; ++t) {
                cacc = __builtin_amdgcn_mfma_f32_16x16x4f32(a4[t].x, cfr[4 * t], cacc, 0, 0, 0);
                f32x4 &c1 = KCM <= 16 ? cacc1 : cacc;
                c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a4[t].y, cfr[4 * t + 1], c1, 0, 0, 0);
                cacc = __builtin_amdgcn_mfma_f32_16x16x4f32(a4[t].z, cfr[4 * t + 2], cacc, 0, 0, 0);
                c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a4[t].w, cfr[4 * t + 3], c1, 0, 0, 0);
            }
            if (KCM <= 16) cacc += cacc1;
            const int col = 16 * cn + c;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = 16 * cm + 4 * g + q;
                Cs[row * LY.CSW + col] = cn < NT ? cacc[q] + (kHold ? lrc : lrs[col]) : 0.f;
            }
          }
        } else if (use_ph) {
            fac_c_ph<BM, KCM>(cb, LY.CBW, phs, A.L, A.lo, A.W, NT, K, lrs, Cs, LY.CSW);
        } else {
            constexpr int MT = BM / 16;
            for (int p = wave; p < MT * NT; p += 8) {
                const int m = p % MT, n = p / MT;
                f32x4 cacc = (f32x4){0.f, 0.f, 0.f, 0.f};
                const float *eb = A.E2 + (int64_t)(16 * n + c) * 2 * K;
#pragma unroll 8
                for (int kk = 0; kk < KCM; ++kk) {
                    const int colk = 4 * kk + g;
                    const float b = colk < 2 * K ? eb[colk] : 0.f;
                    const float a = cb[(16 * m + c) * LY.CBW + colk];
                    cacc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, cacc, 0, 0, 0);
                }
                const int col = 16 * n + c;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int row = 16 * m + 4 * g + q;
                    Cs[row * LY.CSW + col] = cacc[q] + lrs[col];
                }
            }
        }
        lds_barrier();

        // ---- a4 + a5
        const bool short_rows = !WIDE && !(A.flags & (PF_QUERY | PF_LOAD_LSE));
        if (short_rows)
            tile_rows_short<BM, DPT>(A, LY.CSW, Cs, lrs, r0, rows, acc, BFX ? wb : nullptr,
                                     kHold ? &lrhold : nullptr);
        else
            tile_rows<P, BM, DPT>(A, LY.CSW, Cs, lrs, r0, rows, acc);
        if (!(A.flags & PF_ACC_M)) continue;
        lds_barrier();
        if constexpr (BFX) {
            if (!short_rows) {                         // the bf16 planes from the FP32 posteriors
                for (int x = tid; x < BM * 64; x += kThreads) {
                    const int r = x >> 6, i = x & 63;
                    const float w = Cs[r * LY.CSW + i];
                    const __bf16 h = (__bf16)w;
                    ((__bf16 *)(wb + r * 256))[i] = h;
                    ((__bf16 *)(wb + r * 256 + 128))[i] = (__bf16)(w - (float)h);
                }
                lds_barrier();
            }
        }
        tile_wsum<P, DPT>(A, LY.CSW, Cs, rows, acc);
        // (two rows per wave: the M-step applies the row scale from its registers)
        if constexpr (BFX)
            u_fac_bf(wb, ubh, ubl, K, Us, ucol);
        else if constexpr (!WIDE)
            u_fac_reg<BM>(Cs, LY.CSW, ereg, K, RPW == 2 ? nullptr : rowu, Us, ucol);
        else
            if (use_ph)
                u_mfma_ph<BM>(Cs, LY.CSW, phs, A.L, A.lo, A.W, Wp, K, rowu, Us);
            else
                u_mfma<BM>(Cs, LY.CSW, A.E2, Wp, K, rowu, Us);
        lds_barrier();
        // M-step from the rows in registers: this lane's entries over this wave's rows, summed
        // in FP32 over kFacFlush tiles, then the eight waves' partials in wave order into FP64
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            const int j = RPW * rg + r;
            float2 u = j < rows ? Us[j * K + kl] : make_float2(0.f, 0.f);
            if constexpr (!WIDE && RPW == 2) {            // (u_fac_reg left out the row scale)
                u.x *= rsc[r];
                u.y *= rsc[r];
            }
#pragma unroll
            for (int e = 0; e < EPL; ++e) {
                const float2 v = vc[r].entry(e);
                sr[e] = fmaf(u.x, v.x, sr[e]);            // Re (U v)
                sr[e] = fmaf(-u.y, v.y, sr[e]);
                si[e] = fmaf(u.x, v.y, si[e]);            // Im (U v)
                si[e] = fmaf(u.y, v.x, si[e]);
            }
        }
        if (++nacc == (HR ? kFacFlush16 : kFacFlush) || tile + gridDim.x >= ntiles) flush();
    }
    __syncthreads();
    if constexpr (HR) {
#pragma unroll
        for (int cc = 0; cc < DPT; ++cc) {
            const int d = tid + cc * kThreads;
            if (d < D) acc.S[cc] = ((const double2 *)Sw)[d];
        }
        __syncthreads();
    }
    if (A.partials) write_partials(A, acc, smem);
}

// ------------------------------------------------------------------------------------------
// Factored E(+M) pass over a window that is symmetric about offset 0 (the full search on the
// grid, or offsets -h .. h): the offsets +m and -m share the cosines of the rotation phases and
// have sines of opposite sign, so with
//   P_j(m) = sum_k Re c_jk cos(kbar_k theta_m),    Q_j(m) = sum_k Im c_jk sin(kbar_k theta_m)
// the correlations are C_j(+m) = P_j(m) + Q_j(m) and C_j(-m) = P_j(m) - Q_j(m), and
//   Re U_jk = sum_m (w_j(+m) + w_j(-m)) cos(kbar_k theta_m),
//   Im U_jk = sum_m (w_j(+m) - w_j(-m)) sin(kbar_k theta_m)
// (an offset that is its own mirror, 0 or L/2, enters once, with its sines set to 0).  This is the
// factored rewrite of §I eq. (3) with half of its matrix-core products.  Layout: 16-row tiles, two
// rows per wave held in registers (lane l: entries 8 l .. 8 l + 7, D = 512), the next tile's rows
// loading meanwhile; c_jk (scaled by coef s_j) staged in LDS as B fragments; the half-window
// m = 0 .. M - 1 in 16-offset tiles dealt to the waves in turn (wave w: tiles w and w + 8, so
// each SIMD gets the same number), the cosine and sine tables in LDS in A-fragment order.  The
// products run with the window on the matrix rows (C^T = E^T c^T), so each lane holds its row
// j = lane % 16 at four window offsets per tile, and the same registers are the B operand of
// U^T = E w^T (window index 16 t + 4 g + q of lane group g at k-step (t, q)).  Row maxima and sums
// are combined over the waves through LDS in wave order; U^T partials per wave go through LDS and
// are added in wave order by the M-step.  No posterior queries or stored log-sum-exps: those
// passes take the plain factored kernel.

constexpr int kFsWFlush = 16;     // tiles of FP32 W_t partials per FP64 flush

// Geometry of the two forms: E = 8 entries per lane (D = 512, whole rows per wave, 16-row tiles,
// K <= 32) or 16 (D = 2048 in one 16-bit plane, each row over a pair of waves, 8-row tiles,
// K <= 64).  KS: k-steps of 4; TS / CW: row strides (floats) of the cosine / sine tables and of
// the staged c rows, padded so that both products' fragment reads fall in distinct banks; US:
// stride (float2) of a k row of the U^T partials (the M-step's reads, one k per lane pair, then
// fall in distinct banks).
template <int E>
struct FsGeo {
    static constexpr bool HR = E == 16;
    static constexpr int BM = HR ? 8 : 16, RPW = 2, KS = HR ? 16 : 8, KT = KS / 4;
    static constexpr int TS = 4 * KS + 4, CW = 4 * KS + 4, KR = 4 * KS, US = BM + 1;
    static constexpr int NVL = HR ? 128 : 64;
};

struct FsLds {
    int off_ct, off_st, off_lr, off_c, off_x, off_u, off_sw, off_w, off_a, total;
};
template <int E>
__host__ __device__ inline FsLds fs_lds(int MT, int D, int Wp) {
    typedef FsGeo<E> G;
    FsLds l;
    l.off_ct = 0;                                          // cos table, MT x 16 x TS
    l.off_st = l.off_ct + MT * 16 * G::TS * 4;             // sin table
    l.off_lr = l.off_st + MT * 16 * G::TS * 4;             // log rho at +m, then at -m
    l.off_c = l.off_lr + 2 * MT * 16 * 4;                  // Re c rows, then Im c rows
    l.off_x = l.off_c + 2 * 16 * G::CW * 4;                // (max, sum) per wave and row
    l.off_u = l.off_x + 8 * 16 * 8;                        // U^T partials: [wave][k][row] float2
    l.off_sw = l.off_u + 8 * G::KR * G::US * 8;            // M-step partials
    // (E = 8: per wave, FP32, [w][9 (d / 8) + d % 8]; E = 16: one FP64 copy of S)
    l.off_w = align_up(l.off_sw + (G::HR ? D * 16 : 8 * (9 * D / 8) * 8), 16);  // W_t (FP64)
    l.off_a = align_up(l.off_w + Wp * 8, 16);              // a (FP32), lane-major
    l.total = l.off_a + D * 8;
    return l;
}

// The half window (lo taken mod L): W = L (the full search, any lo) or W = 2 h + 1 with
// lo = -h mod L (offsets -h .. h).  M offsets m = 0 .. M - 1; fs_plus(m) is the window index of
// offset +m, fs_mirror(m) that of -m, or -1 when -m is +m itself (m = 0, or L / 2 for even L).
__host__ __device__ inline int fs_halves(int L, int lo, int W) {
    return W == L ? L / 2 + 1 : (W + 1) / 2;
}
__host__ __device__ inline int fs_mod(int x, int L) {
    const int r = x % L;
    return r < 0 ? r + L : r;
}
__host__ __device__ inline int fs_plus(int m, int L, int lo) { return fs_mod(m - lo, L); }
__host__ __device__ inline int fs_mirror(int m, int L, int lo, int W) {
    const int i = fs_mod(-m - lo, L);
    return (i < W && i != fs_plus(m, L, lo)) ? i : -1;
}
// The same for 0 <= m < L and 0 <= lo < L without a division (the kernels' tables)
__device__ __forceinline__ int fs_plus_d(int m, int L, int lo) {
    const int x = m - lo;
    return x < 0 ? x + L : x;
}
__device__ __forceinline__ int fs_mirror_d(int m, int L, int lo, int W) {
    int i = L - m - lo;                            // in (-L, L]
    i = i < 0 ? i + L : (i == L ? 0 : i);
    return (i < W && i != fs_plus_d(m, L, lo)) ? i : -1;
}

template <int P, int MTW, int E>
__global__ __launch_bounds__(kThreads) void pass_fs_kernel(PassArgs A) {
    typedef FsGeo<E> G;
    constexpr bool HR = G::HR;
    constexpr int EPL = E, RPW = G::RPW, BM = G::BM, KS = G::KS, KT = G::KT;
    constexpr int TS = G::TS, CW = G::CW, KR = G::KR, US = G::US, NVL = G::NVL;
    constexpr int DPT = NVL * EPL / kThreads;          // S entries per thread (1 or 4)
    static_assert(!HR || P == P_F16 || P == P_BF16, "rows over wave pairs: one 16-bit plane");
    if ((A.flags & PF_CHECK_STOP) && *A.stopped) return;

    extern __shared__ __align__(16) uint8_t smem[];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int g = lane >> 4, c16 = lane & 15;
    const int K = A.K, D = A.D, L = A.L, lo = A.lo, W = A.W, Wp = A.Wp;
    const int M = fs_halves(L, lo, W), MT = (M + 15) / 16;
    const FsLds LY = fs_lds<E>(MT, D, Wp);
    const int hh = HR ? (wave & 1) : 0, rg = HR ? (wave >> 1) : wave;   // half, row group
    const int vl = 64 * hh + lane;                 // this lane's place in the row
    float *ct = (float *)(smem + LY.off_ct);
    float *st = (float *)(smem + LY.off_st);
    float *lrp = (float *)(smem + LY.off_lr);
    float *lrm = lrp + MT * 16;
    float *cs = (float *)(smem + LY.off_c);
    float2 *xs = (float2 *)(smem + LY.off_x);
    float2 *up = (float2 *)(smem + LY.off_u);
    float2 *Sw = (float2 *)(smem + LY.off_sw);
    double *wt64 = (double *)(smem + LY.off_w);
    float2 *as = (float2 *)(smem + LY.off_a);

    // tables: ct / st entry [m][k] (row stride TS) = cos / sin (kbar_k theta_m) (zero past M
    // and K; sines zero where the offset is its own mirror).  Wave w fills rows w, w + 8, ...,
    // lane l entry k = l (K <= 64; entries 64 .. TS - 1 are zero); a row's window indices are
    // uniform over the wave, and 24 rows' reads (all of a wave's rows up to M = 192) are issued
    // before any is stored.
    static_assert(TS - 64 <= 64, "one extra lane pass of zeros");
    constexpr int RU = 24;
    for (int m0 = wave; m0 < MT * 16; m0 += 8 * RU) {
        float cv[RU], sv[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int m = m0 + 8 * u;
            const bool ok = m < M && lane < K;
            const int ip = m < M ? fs_plus_d(m, L, lo) : 0;
            const bool mir = m < M && fs_mirror_d(m, L, lo, W) >= 0;
            const float *e = A.E2 + (int64_t)ip * 2 * K;
            const float c0 = e[ok ? lane : 0], s0 = e[ok ? K + lane : 0];
            cv[u] = ok ? c0 : 0.f;
            sv[u] = ok && mir ? s0 : 0.f;
        }
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int m = m0 + 8 * u;
            if (m < MT * 16) {
                if (lane < TS) {
                    ct[m * TS + lane] = cv[u];
                    st[m * TS + lane] = sv[u];
                }
                if (64 + lane < TS) {
                    ct[m * TS + 64 + lane] = 0.f;
                    st[m * TS + 64 + lane] = 0.f;
                }
            }
        }
    }
    for (int m = tid; m < MT * 16; m += kThreads) {
        float p = -INFINITY, q = -INFINITY;
        if (m < M) {
            p = A.logrho32[fs_plus_d(m, L, lo)];
            const int im = fs_mirror_d(m, L, lo, W);
            if (im >= 0) q = A.logrho32[im];
        }
        lrp[m] = p;
        lrm[m] = q;
    }
    // c rows past the tile's rows and columns k >= K stay zero
    for (int x = tid; x < 2 * 16 * CW; x += kThreads) cs[x] = 0.f;
    // the exchange slots of waves without window tiles keep (-inf, 0) and zero U partials
    for (int x = tid; x < 8 * 16; x += kThreads) xs[x] = make_float2(-INFINITY, 0.f);
    for (int x = tid; x < 8 * KR * US; x += kThreads) up[x] = make_float2(0.f, 0.f);
    for (int i = tid; i < Wp; i += kThreads) wt64[i] = 0.0;
    {
        constexpr int NA = NVL * EPL / kThreads;        // D <= NVL EPL entries, read together
        double2 av[NA];
#pragma unroll
        for (int c = 0; c < NA; ++c) {
            const int d = tid + c * kThreads;
            av[c] = d < D ? ((const double2 *)A.a)[d] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int c = 0; c < NA; ++c) {
            const int d = tid + c * kThreads;
            if (d < D) as[(d % EPL) * NVL + d / EPL] = make_float2((float)av[c].x, (float)av[c].y);
        }
    }
    if constexpr (HR)
        for (int d = tid; d < D; d += kThreads) ((double2 *)Sw)[d] = make_double2(0.0, 0.0);
    __syncthreads();

    const int kl = EPL * vl / A.Q;                 // this lane's angular frequency index
    const int LPK = A.Q / EPL;
    float lpk_f[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) lpk_f[t] = LPK > (1 << t) ? 1.f : 0.f;
    const float coef = (float)A.coef;
    const int nwu = MT < 8 ? MT : 8;                // waves holding window tiles

    PassAcc<DPT> acc;
    acc.init();
    const int64_t ntiles = (A.row_end - A.row_begin + BM - 1) / BM;
    FacRow<P, EPL> vn[RPW];
    float rsn[RPW];
    auto load_tile = [&](int64_t t) {
        const int64_t rb = A.row_begin + t * BM + RPW * rg;
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            const int64_t row = rb + r < A.row_end ? rb + r : A.row_end - 1;
            // (the second half of a split row starts after D/2 entries of 4 bytes)
            vn[r].load(A.V + row * A.rowbytes + (HR ? hh * (D / 2) * 4 : 0), A.Dp, lane);
            rsn[r] = A.rowscale ? A.rowscale[row] : 1.0f;
        }
    };
    float sr[EPL], si[EPL];
#pragma unroll
    for (int e = 0; e < EPL; ++e) sr[e] = si[e] = 0.f;
    int nacc = 0;
    auto flush_s = [&]() {
      if constexpr (HR) {
        // the four row groups add their FP32 partials into the FP64 copy of S in order (the two
        // halves of a group own disjoint entries)
        double2 *Sd = (double2 *)Sw;
        const int d0 = EPL * vl;
        for (int w = 0; w < 4; ++w) {
            if (rg == w)
#pragma unroll
                for (int e = 0; e < EPL; ++e) {
                    double2 t = Sd[d0 + e];
                    t.x += (double)sr[e];
                    t.y += (double)si[e];
                    Sd[d0 + e] = t;
                }
            lds_barrier();
        }
      } else {
        // wave w's partials at [w][9 (d / 8) + d % 8], then summed in wave order per entry
        constexpr int SWS = 9 * 512 / 8;                   // (D = 512)
#pragma unroll
        for (int e = 0; e < EPL; ++e) Sw[wave * SWS + 9 * lane + e] = make_float2(sr[e], si[e]);
        lds_barrier();
        {
            const int d = tid;
            const int o = 9 * (d >> 3) + (d & 7);
            float2 s = Sw[o];
#pragma unroll
            for (int w = 1; w < 8; ++w) {
                const float2 t = Sw[w * SWS + o];
                s.x += t.x;
                s.y += t.y;
            }
            acc.S[0].x += (double)s.x;
            acc.S[0].y += (double)s.y;
        }
      }
#pragma unroll
        for (int e = 0; e < EPL; ++e) sr[e] = si[e] = 0.f;
        nacc = 0;
    };
    // this lane's W_t partials (its row j = c16, its window offsets), FP32 over kFsWFlush tiles;
    // the flush sums the 16 rows by DPP and adds them in FP64 (each offset has one owner lane)
    float wsp[MTW][4], wsm[MTW][4];
#pragma unroll
    for (int t = 0; t < MTW; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) wsp[t][q] = wsm[t][q] = 0.f;
    int nw = 0;
    auto flush_w = [&]() {
#pragma unroll
        for (int t = 0; t < MTW; ++t) {
            const int mt = wave + 8 * t;
            if (mt >= MT) break;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float sp = row16_sum(wsp[t][q]), sm = row16_sum(wsm[t][q]);
                const int m = 16 * mt + 4 * g + q;
                if (c16 == 0 && m < M) {
                    wt64[fs_plus_d(m, L, lo)] += (double)sp;
                    const int im = fs_mirror_d(m, L, lo, W);
                    if (im >= 0) wt64[im] += (double)sm;
                }
                wsp[t][q] = wsm[t][q] = 0.f;
            }
        }
        nw = 0;
    };
    double wc_acc = 0.0;

    int64_t tile = blockIdx.x;
    if (tile < ntiles) load_tile(tile);
    for (; tile < ntiles; tile += gridDim.x) {
        const int64_t r0 = A.row_begin + tile * BM;
        const int rows = (int)((A.row_end - r0) < BM ? (A.row_end - r0) : BM);
        FacRow<P, EPL> vc[RPW];
        float rsc[RPW];
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            vc[r] = vn[r];
            rsc[r] = rsn[r];
        }
        const bool pf = tile + gridDim.x < ntiles;
        if (pf && wave < 4) load_tile(tile + gridDim.x);

        // ---- c_jk of this wave's rows, scaled by coef s_j, into the B-fragment staging (the
        // lane's coefficients read from LDS once per tile)
        float2 areg[EPL];
#pragma unroll
        for (int e = 0; e < EPL; ++e) areg[e] = as[e * NVL + vl];
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            const int j = RPW * rg + r;
            float cr = 0.f, ci = 0.f;
#pragma unroll
            for (int e = 0; e < EPL; ++e) {
                const float2 v = vc[r].entry(e);
                cr = fmaf(v.x, areg[e].x, cr);            // Re conj(v) a
                cr = fmaf(v.y, areg[e].y, cr);
                ci = fmaf(v.x, areg[e].y, ci);            // Im conj(v) a
                ci = fmaf(-v.y, areg[e].x, ci);
            }
            cr = lanes_sum_dpp(cr, lpk_f);
            ci = lanes_sum_dpp(ci, lpk_f);
            for (int o = 16; o < LPK; o <<= 1) {
                cr += __shfl_xor(cr, o);
                ci += __shfl_xor(ci, o);
            }
            const float u = j < rows ? rsc[r] : 1.0f;
            if ((lane & (LPK - 1)) == 0) {
                const int o = j * CW + (kl & 3) * KS + (kl >> 2);
                cs[o] = cr * (coef * u);
                cs[16 * CW + o] = ci * (coef * u);
            }
        }
        lds_barrier();
        if (pf && wave >= 4) load_tile(tile + gridDim.x);

        // ---- P^T and Q^T for this wave's window tiles; log-weights at +m and -m
        // B fragments of k-step ks: c[j = lane % 16][4 ks + lane / 16], KS consecutive floats
        const float4 *pbr = (const float4 *)(cs + c16 * CW + KS * g);
        const float4 *pbi = (const float4 *)(cs + 16 * CW + c16 * CW + KS * g);
        float lp[MTW][4], lm[MTW][4];
        float mloc = -INFINITY;
#pragma unroll
        for (int t = 0; t < MTW; ++t) {
            const int mt = wave + 8 * t;
            if (mt >= MT) {
#pragma unroll
                for (int q = 0; q < 4; ++q) lp[t][q] = lm[t][q] = -INFINITY;
                continue;
            }
            f32x4 pa = (f32x4){0.f, 0.f, 0.f, 0.f}, qa = pa;
            // A fragment of k-step ks: offset m = 16 mt + lane % 16, k = 4 ks + lane / 16
            const float *ca = ct + (16 * mt + c16) * TS + g;
            const float *sa = st + (16 * mt + c16) * TS + g;
#pragma unroll
            for (int k4 = 0; k4 < KS / 4; ++k4) {
                const float4 b4r = pbr[k4], b4i = pbi[k4];
                const float brv[4] = {b4r.x, b4r.y, b4r.z, b4r.w};
                const float biv[4] = {b4i.x, b4i.y, b4i.z, b4i.w};
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int ks = 4 * k4 + u;
                    pa = __builtin_amdgcn_mfma_f32_16x16x4f32(ca[4 * ks], brv[u], pa, 0, 0, 0);
                    qa = __builtin_amdgcn_mfma_f32_16x16x4f32(sa[4 * ks], biv[u], qa, 0, 0, 0);
                }
            }
            const float4 lp4 = *(const float4 *)(lrp + 16 * mt + 4 * g);
            const float4 lm4 = *(const float4 *)(lrm + 16 * mt + 4 * g);
            const float lpv[4] = {lp4.x, lp4.y, lp4.z, lp4.w};
            const float lmv[4] = {lm4.x, lm4.y, lm4.z, lm4.w};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                lp[t][q] = (pa[q] + qa[q]) + lpv[q];
                lm[t][q] = (pa[q] - qa[q]) + lmv[q];
                mloc = fmaxf(mloc, fmaxf(lp[t][q], lm[t][q]));
            }
        }
        // this wave's maximum and sum for row j over the four lane groups; its exponentials,
        // relative to that maximum, are the B operand of the U^T product (the row's factor
        // exp(m_wave - m_row) / sum, a column scale of U^T, is applied after the exchange).  With
        // 8 entries per lane the products run before the exchange, beside the exponentials; with
        // 16 (the rows and M-step sums take twice the registers) after it.
        mloc = fmaxf(mloc, swz_xor16(mloc));
        mloc = fmaxf(mloc, __shfl_xor(mloc, 32));
        const bool accm = (A.flags & PF_ACC_M) != 0;
        float ep[MTW][4], em[MTW][4], sloc = 0.f, wcl = 0.f;
        f32x4 ur[KT], ui[KT];
#pragma unroll
        for (int kt = 0; kt < KT; ++kt) ur[kt] = ui[kt] = (f32x4){0.f, 0.f, 0.f, 0.f};
        // U^T = E e^T over window tile t (Re: cos with e(+m) + e(-m); Im: sin with e(+m) - e(-m));
        // A fragment: k = 16 kt + lane % 16, offset m = 16 mt + 4 g + q
        auto u_tile = [&](int t) {
            const int mt = wave + 8 * t;
            if (!accm || mt >= MT) return;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float ws = ep[t][q] + em[t][q], wd = ep[t][q] - em[t][q];
#pragma unroll
                for (int kt = 0; kt < KT; ++kt) {
                    const int o = (16 * mt + 4 * g + q) * TS + 16 * kt + c16;
                    ur[kt] = __builtin_amdgcn_mfma_f32_16x16x4f32(ct[o], ws, ur[kt], 0, 0, 0);
                    ui[kt] = __builtin_amdgcn_mfma_f32_16x16x4f32(st[o], wd, ui[kt], 0, 0, 0);
                }
            }
        };
#pragma unroll
        for (int t = 0; t < MTW; ++t) {
            const int mtl = (wave + 8 * t) < MT ? wave + 8 * t : 0;
            const float4 lp4 = *(const float4 *)(lrp + 16 * mtl + 4 * g);
            const float4 lm4 = *(const float4 *)(lrm + 16 * mtl + 4 * g);
            const float lpv[4] = {lp4.x, lp4.y, lp4.z, lp4.w};
            const float lmv[4] = {lm4.x, lm4.y, lm4.z, lm4.w};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                // (the exponentials and sum_i e_ji (l_ji - log rho_i), both relative to m_wave)
                const bool fp = lp[t][q] != -INFINITY, fm = lm[t][q] != -INFINITY;
                ep[t][q] = fp ? __expf(lp[t][q] - mloc) : 0.f;
                em[t][q] = fm ? __expf(lm[t][q] - mloc) : 0.f;
                sloc += ep[t][q] + em[t][q];
                if (fp) wcl = fmaf(ep[t][q], lp[t][q] - lpv[q], wcl);
                if (fm) wcl = fmaf(em[t][q], lm[t][q] - lmv[q], wcl);
            }
            if constexpr (!HR) u_tile(t);
        }
        sloc += swz_xor16(sloc);
        sloc += __shfl_xor(sloc, 32);
        if (g == 0 && wave < nwu) xs[wave * 16 + c16] = make_float2(mloc, sloc);
        lds_barrier();

        // ---- posteriors: the row's maximum and sum over the waves, in wave order
        float2 xw[8];
#pragma unroll
        for (int w = 0; w < 8; ++w) xw[w] = xs[w * 16 + c16];
        float gmax = xw[0].x;
#pragma unroll
        for (int w = 1; w < 8; ++w) gmax = fmaxf(gmax, xw[w].x);
        float tot = 0.f;
#pragma unroll
        for (int w = 0; w < 8; ++w) tot += xw[w].y > 0.f ? xw[w].y * __expf(xw[w].x - gmax) : 0.f;
        const bool valid = c16 < rows;
        const float scale = (valid && sloc > 0.f) ? __expf(mloc - gmax) / tot : 0.f;
#pragma unroll
        for (int t = 0; t < MTW; ++t) {
            if (wave + 8 * t >= MT) break;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                wsp[t][q] = fmaf(ep[t][q], scale, wsp[t][q]);
                wsm[t][q] = fmaf(em[t][q], scale, wsm[t][q]);
            }
        }
        wc_acc += (double)(wcl * scale);          // sum_i w_ji (l_ji - log rho_i), this lane's
        if (wave == 0 && g == 0 && valid) {
            acc.lse += (double)(gmax + __logf(tot));
            acc.rows += 1.0;
        }
        if (++nw == kFsWFlush) flush_w();
        if (!accm) continue;
        if constexpr (HR) {
            // two column tiles of U^T at a time (half the accumulators live), each written out
            // before the next pair
            static_assert(MTW == 1, "one window tile per wave");
            const int mt = wave;
#pragma unroll
            for (int kp = 0; kp < KT; kp += 2) {
                f32x4 u2r[2], u2i[2];
#pragma unroll
                for (int h = 0; h < 2; ++h) u2r[h] = u2i[h] = (f32x4){0.f, 0.f, 0.f, 0.f};
                if (mt < MT) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const float ws = ep[0][q] + em[0][q], wd = ep[0][q] - em[0][q];
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            const int o = (16 * mt + 4 * g + q) * TS + 16 * (kp + h) + c16;
                            u2r[h] = __builtin_amdgcn_mfma_f32_16x16x4f32(ct[o], ws, u2r[h], 0, 0, 0);
                            u2i[h] = __builtin_amdgcn_mfma_f32_16x16x4f32(st[o], wd, u2i[h], 0, 0, 0);
                        }
                    }
                }
                if (wave < nwu && c16 < BM) {
#pragma unroll
                    for (int h = 0; h < 2; ++h)
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            up[(wave * KR + 16 * (kp + h) + 4 * g + q) * US + c16] =
                                make_float2(u2r[h][q] * scale, u2i[h][q] * scale);
                }
            }
        } else if (wave < nwu) {
#pragma unroll
            for (int kt = 0; kt < KT; ++kt)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    up[(wave * KR + 16 * kt + 4 * g + q) * US + c16] =
                        make_float2(ur[kt][q] * scale, ui[kt][q] * scale);
        }
        lds_barrier();

        // ---- M-step from the rows in registers: U_jk summed over the waves in wave order, times
        // the row scale; this lane's entries over this wave's rows, FP32 over kFacFlush tiles
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            const int j = RPW * rg + r;
            float2 u = make_float2(0.f, 0.f);
            if (j < rows) {
                float2 ut[8];
#pragma unroll
                for (int w = 0; w < 8; ++w) ut[w] = up[(w * KR + kl) * US + j];
#pragma unroll
                for (int w = 0; w < 8; ++w) {
                    u.x += ut[w].x;
                    u.y += ut[w].y;
                }
                u.x *= rsc[r];
                u.y *= rsc[r];
            }
#pragma unroll
            for (int e = 0; e < EPL; ++e) {
                const float2 v = vc[r].entry(e);
                sr[e] = fmaf(u.x, v.x, sr[e]);            // Re (U v)
                sr[e] = fmaf(-u.y, v.y, sr[e]);
                si[e] = fmaf(u.x, v.y, si[e]);            // Im (U v)
                si[e] = fmaf(u.y, v.x, si[e]);
            }
        }
        if (++nacc == (HR ? kFacFlush16 : kFacFlush) || tile + gridDim.x >= ntiles) flush_s();
    }
    if (nw) flush_w();
    __syncthreads();
    if constexpr (HR) {
#pragma unroll
        for (int cc = 0; cc < DPT; ++cc) acc.S[cc] = ((const double2 *)Sw)[tid + cc * kThreads];
    }
    acc.wc = wc_acc;
    for (int c = 0; c < 2; ++c) {
        const int i = tid + c * kThreads;
        if (i < Wp) acc.W[c] = i < W ? wt64[i] : 0.0;
    }
    __syncthreads();
    if (A.partials) write_partials(A, acc, smem);
}

// ------------------------------------------------------------------------------------------
// a6: FP64 reduction of the workgroup partials (kRedCols columns per workgroup, all G rows in a
// fixed order), then the FP64 finalize in the workgroup that finishes last (one launch).

constexpr int kFinThreads = 512;
constexpr int kFinWaves = kFinThreads / 64;
constexpr int kRedCols = 8;                        // partial columns per reducing workgroup

// FP64 lane exchanges by DPP on the two 32-bit halves (no LDS round trip), and a lane's value
// read by every lane of the wave.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double rl_d(double v, int lane) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_readlane((int)(unsigned)u, lane);
    const int hi = __builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
template <int OP>
__device__ __forceinline__ double fin_op(double a, double b) {
    return OP ? fmax(a, b) : a + b;
}
// Sum (OP = 0) or maximum (OP = 1) over each 16-lane row (xor 1, xor 2, half-mirror, mirror:
// every lane of the row ends with the same value), then over the wave (rows 0..3 read in order).
// Every lane must be active.
template <int OP>
__device__ __forceinline__ double row16_reduce_d(double v) {
    v = fin_op<OP>(v, dpp_d<0xB1>(v));
    v = fin_op<OP>(v, dpp_d<0x4E>(v));
    v = fin_op<OP>(v, dpp_d<0x141>(v));
    return fin_op<OP>(v, dpp_d<0x140>(v));
}
template <int OP>
__device__ __forceinline__ double wave_reduce_d(double v) {
    v = row16_reduce_d<OP>(v);
    return fin_op<OP>(fin_op<OP>(rl_d(v, 0), rl_d(v, 16)), fin_op<OP>(rl_d(v, 32), rl_d(v, 48)));
}

// Deterministic workgroup sums (OP = 0) or maxima (OP = 1) of NV doubles per thread: a fixed-order
// reduction over the wave's 64 lanes (every lane ends with the same value), then the kFinWaves
// wave results in wave order.  sh holds NV x kFinWaves doubles; every thread must call it.
template <int NV, int OP = 0>
__device__ __forceinline__ void fin_block_reduce(double (&v)[NV], double *sh) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_reduce_d<OP>(v[k]);
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) sh[k * kFinWaves + wave] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double t = sh[k * kFinWaves];
        for (int w = 1; w < kFinWaves; ++w) t = fin_op<OP>(t, sh[k * kFinWaves + w]);
        v[k] = t;
    }
}
// One maximum and one sum in the same pass (one pair of barriers).
__device__ __forceinline__ void fin_block_max_sum(double &mx, double &sm, double *sh) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    mx = wave_reduce_d<1>(mx);
    sm = wave_reduce_d<0>(sm);
    __syncthreads();
    if (lane == 0) {
        sh[wave] = mx;
        sh[kFinWaves + wave] = sm;
    }
    __syncthreads();
    double a = sh[0], b = sh[kFinWaves];
    for (int w = 1; w < kFinWaves; ++w) {
        a = fmax(a, sh[w]);
        b += sh[kFinWaves + w];
    }
    mx = a;
    sm = b;
}

// A reduced sum, read at device scope: the other workgroups of the reducing launch wrote it with
// device-scope stores, so the read skips this CU's caches.
__device__ __forceinline__ double ld_red(const double *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The finalize proper (one workgroup), on the reduced sums in F.red.
__device__ void finalize_body(const FinArgs &F) {
    __shared__ double sh[8 * kFinWaves];
    __shared__ double2 anew[kMaxD];
    __shared__ double2 ain[kMaxD];
    __shared__ double2 ck[kMaxK];
    const int t = threadIdx.x;
    const int D = F.D, W = F.W, K = F.K, L = F.L;
    const double N = (double)F.N;
    const double *S = F.red;
    const double *Wt = F.red + 2 * D;
    const double s_lse = ld_red(F.red + 2 * D + F.Wp);
    const double s_wc = ld_red(F.red + 2 * D + F.Wp + 1);

    if (F.mode != FIN_EM) {
        double v[1] = {0.0};
        for (int r = t; r < 2 * D; r += kFinThreads) v[0] += F.a_in[r] * F.a_in[r];
        fin_block_reduce<1>(v, sh);
        const double an2 = v[0];
        const double ll = s_lse - (F.sum_vn2 + N * an2) / F.sigma2 -
                          N * (double)D * log(M_PI * F.sigma2);
        if (F.mode == FIN_LL) {
            if (t == 0) F.out[0] = ll;
            return;
        }
        const double c = F.g * 2.0 / F.sigma2;
        for (int r = t; r < 2 * D; r += kFinThreads)
            F.grad_a[r] = c * (ld_red(S + r) - N * F.a_in[r]);
        if (F.grad_eta)
            for (int i = t; i < W; i += kFinThreads)
                F.grad_eta[i] = F.g * (ld_red(Wt + i) - N * F.rho_in[i]);
        if (t == 0) {
            const double swr = F.sum_vn2 + N * an2 - 2.0 * s_wc;
            F.out[0] = ll;
            F.out[1] = F.g * (-N * (double)D / F.sigma2 + swr / (F.sigma2 * F.sigma2));
        }
        return;
    }

    // FIN_EM.  Every input (a_t, S, the prior terms, W_t, the first phase, t, the stop flag) is
    // loaded up front, so the workgroup waits on global memory once.
    constexpr int DPF = kMaxD / kFinThreads, WPF = kMaxWp / kFinThreads;
    const double2 ph0 = t < L ? F.phase[t] : make_double2(1.0, 0.0);
    double2 at[DPF], sd[DPF];
    double gv[DPF];
#pragma unroll
    for (int c = 0; c < DPF; ++c) {
        const int d = t + c * kFinThreads;
        at[c] = sd[c] = make_double2(0.0, 0.0);
        gv[c] = 0.0;
        if (d < D) {
            at[c] = ((const double2 *)F.a_in)[d];
            sd[c] = make_double2(ld_red(S + 2 * d), ld_red(S + 2 * d + 1));
            if (F.gai) gv[c] = F.gai[d];
        }
    }
    // rho entries i = tw, tw + kFinThreads, ... with tw = (t + 128) mod kFinThreads: windows up
    // to 128 land on the last two waves, which have no rotation of the stopping metric (L <= 384),
    // so that their logarithms run beside it
    const int tw = (t + 128) % kFinThreads;
    double wt[WPF], rb[WPF], ri[WPF];
#pragma unroll
    for (int c = 0; c < WPF; ++c) {
        const int i = tw + c * kFinThreads;
        wt[c] = rb[c] = 0.0;
        ri[c] = 1.0;
        if (i < W) {
            wt[c] = ld_red(Wt + i);
            rb[c] = F.rho_bar[i];
            ri[c] = F.rho_in[i];
        }
    }
    const int64_t it = *F.t;
    if (*F.stopped) return;

    // ||a_t||^2, MAP prior terms, a_{t+1}, ||a_{t+1}||^2, ||a_{t+1} - a_t||^2, the rho normaliser
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double2 an[DPF];
    const double rden0 = 1.0 / N;                 // (the same as below with no prior on a)
#pragma unroll
    for (int c = 0; c < DPF; ++c) {
        const int d = t + c * kFinThreads;
        const double rden = F.gai ? 1.0 / (N + F.sigma2 * gv[c]) : rden0;
        an[c] = make_double2(sd[c].x * rden, sd[c].y * rden);
        if (d < D) {
            const double ar = at[c].x, ai = at[c].y;
            anew[d] = an[c];
            ain[d] = at[c];
            v[0] += ar * ar + ai * ai;
            v[1] -= gv[c] * (ar * ar + ai * ai);
            v[2] += an[c].x * an[c].x + an[c].y * an[c].y;
            v[3] += (an[c].x - ar) * (an[c].x - ar) + (an[c].y - ai) * (an[c].y - ai);
        }
    }
#pragma unroll
    for (int c = 0; c < WPF; ++c) {
        if (tw + c * kFinThreads >= W) continue;
        if (F.gamma != 0.0 && rb[c] > 0.0) v[1] += F.gamma * rb[c] * log(ri[c]);
        v[4] += wt[c] + F.gamma * rb[c];
    }
    fin_block_reduce<5>(v, sh);                 // its barriers also publish anew, ain, ph
    const double an2 = v[0], jprior = v[1], nn2 = v[2], dl2 = v[3], tot = v[4];
    const double ll = s_lse - (F.sum_vn2 + N * an2) / F.sigma2 -
                      N * (double)D * log(M_PI * F.sigma2);

    // c_k = sum_q conj(a_new[k,q]) a_t[k,q]: 16 lanes per k (q = lane % 16, + 16, ...), their
    // partial sums combined inside the 16-lane DPP row
    for (int k0 = 0; k0 < K; k0 += kFinThreads / 16) {
        const int k = k0 + t / 16, qp = t % 16;
        double cr = 0.0, ci = 0.0;
        if (k < K)
            for (int q = qp; q < F.Q; q += 16) {
                const int d = k * F.Q + q;
                const double2 a1 = anew[d], a0 = ain[d];
                cr += a1.x * a0.x + a1.y * a0.y;
                ci += a1.x * a0.y - a1.y * a0.x;
            }
        cr = row16_reduce_d<0>(cr);
        ci = row16_reduce_d<0>(ci);
        if (k < K && qp == 0) ck[k] = make_double2(cr, ci);
    }
    __syncthreads();
    // rho_{t+1}, its log (-inf on zero entries and on the padding up to Wp) and a_{t+1}, stored
    // at once (nothing below changes them)
    const double rtot = 1.0 / tot;
    double ent = 0.0;
#pragma unroll
    for (int c = 0; c < WPF; ++c) {
        const int i = tw + c * kFinThreads;
        if (i >= F.Wp) continue;
        const double r = i < W ? (F.update_rho ? (wt[c] + F.gamma * rb[c]) * rtot : ri[c]) : 0.0;
        const double l = r > 0.0 ? log(r) : -INFINITY;
        if (r > 0.0) ent -= r * l;
        if (i < W && F.update_rho) F.rho[i] = r;
        F.logrho32[i] = (float)l;
        F.logrho64[i] = l;
    }
#pragma unroll
    for (int c = 0; c < DPF; ++c) {
        const int d = t + c * kFinThreads;
        if (d < D) ((double2 *)F.a)[d] = an[c];
    }
    // stopping metric min_l ||a_new - exp(-2 pi i kbar l / L) a_t||^2: Re sum_k c_k z^k at
    // z = exp(-2 pi i l / L), one rotation per thread, as four interleaved Horner chains in z^4
    // (p = h_0 + z (h_1 + z (h_2 + z h_3)), h_r = sum_j c_{4j+r} z^{4j}); |z| = 1, so the rounding
    // error stays within a few K eps sum_k |c_k|
    double best = INFINITY;
    const int J = (K + 3) / 4;
    for (int l = t; l < L; l += kFinThreads) {
        const double2 p = l == t ? ph0 : F.phase[l];          // exp(+2 pi i l / L)
        const double zx = p.x, zy = -p.y;
        const double z2x = zx * zx - zy * zy, z2y = 2.0 * zx * zy;
        const double wx = z2x * z2x - z2y * z2y, wy = 2.0 * z2x * z2y;
        double hx[4], hy[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int k = 4 * (J - 1) + r;
            hx[r] = k < K ? ck[k].x : 0.0;
            hy[r] = k < K ? ck[k].y : 0.0;
        }
        for (int j = J - 2; j >= 0; --j) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const double2 c = ck[4 * j + r];
                const double nx = fma(hx[r], wx, fma(-hy[r], wy, c.x));
                hy[r] = fma(hx[r], wy, fma(hy[r], wx, c.y));
                hx[r] = nx;
            }
        }
        double px = hx[3], py = hy[3];
#pragma unroll
        for (int r = 2; r >= 0; --r) {
            const double nx = fma(px, zx, fma(-py, zy, hx[r]));
            py = fma(px, zy, fma(py, zx, hy[r]));
            px = nx;
        }
        best = fmin(best, nn2 + an2 - 2.0 * px);
    }
    {
        double mx = -best;
        fin_block_max_sum(mx, ent, sh);
        best = -mx;
    }
    if (t == 0) {
        double *rec = F.stats + (it % kStatsCap) * 6;
        rec[0] = (double)it;
        rec[1] = ll;
        rec[2] = ll + jprior;
        rec[3] = dl2;
        rec[4] = best;
        rec[5] = ent;
        *F.ll_last = ll;
        *F.t = it + 1;
        if (F.tol > 0.0 && best < F.tol) *F.stopped = 1;
    }
}

// Fixed-order FP64 sum of a pass's partials: workgroup b sums columns [8 b, 8 b + 8) over the G
// rows.  Thread t = 8 g + c takes column c of rows g, g + 64, ...; the eight row groups of a wave
// are combined by a butterfly (lanes 8 apart, then 16, then 32), then the eight waves in order.  Each
// workgroup then counts itself done on *count (atomicInc wraps it back to 0 on the last one, so
// no clearing is needed between launches); the last runs the finalize on the sums.  With the
// stop flag set every workgroup leaves before counting.
__global__ __launch_bounds__(kFinThreads) void reduce_finalize_kernel(FinArgs F,
                                                                      const double *partials,
                                                                      int G, int ncols,
                                                                      double *red,
                                                                      unsigned *count) {
    __shared__ double rsh[kFinWaves * kRedCols];
    __shared__ int last;
    constexpr int NG = kFinThreads / kRedCols;
    static_assert(kRedCols == 8 && NG == 64, "row groups: 8 per wave");
    const int t = threadIdx.x, cl = t % kRedCols, gs = t / kRedCols, wave = t >> 6;
    const int col = blockIdx.x * kRedCols + cl;
    double s = 0.0;
    if (col < ncols) {
#pragma unroll 8
        for (int b = gs; b < G; b += NG) s += partials[(int64_t)b * ncols + col];
    }
    s += __shfl_xor(s, 8);
    s += __shfl_xor(s, 16);
    s += __shfl_xor(s, 32);
    if (F.mode == FIN_EM && *F.stopped) return;
    if ((t & 63) < kRedCols) rsh[wave * kRedCols + cl] = s;
    __syncthreads();
    if (t < kRedCols && col < ncols) {
        double u = rsh[t];
#pragma unroll
        for (int w = 1; w < kFinWaves; ++w) u += rsh[w * kRedCols + t];
        __hip_atomic_store(red + col, u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // The sums are device-scope stores (written through to the device's coherence point, so no
    // cache write-back is needed); the workgroup counts itself done once they have completed, and
    // the last one reads them back with device-scope loads.
    wait_vm<0>();
    __syncthreads();
    if (t == 0) last = atomicInc(count, gridDim.x - 1) == gridDim.x - 1;
    __syncthreads();
    if (!last) return;
    finalize_body(F);
}

// ------------------------------------------------------------------------------------------
// a8: histogram of integer rotation errors (mod L).

__global__ __launch_bounds__(256) void histogram_kernel(const int32_t *err, int64_t n, int L,
                                                        unsigned long long *counts) {
    extern __shared__ unsigned int bins[];
    for (int i = threadIdx.x; i < L; i += 256) bins[i] = 0u;
    __syncthreads();
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * 256) {
        int b = err[p] % L;
        if (b < 0) b += L;
        atomicAdd(&bins[b], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < L; i += 256)
        if (bins[i]) atomicAdd(&counts[i], (unsigned long long)bins[i]);
}

// ------------------------------------------------------------------------------------------
// launchers

hipError_t launch_convert(int prec, const void *obs, int64_t N, int D, int Dp, uint8_t *V,
                          int64_t rowbytes, float *rowscale, double *vnorm2, int *nonfinite,
                          hipStream_t s) {
    int64_t blocks = (N + 3) / 4;
    if (blocks > 65536) blocks = 65536;
    dim3 g((unsigned)blocks), b(256);
    switch (prec) {
    case P_F64:
        hipLaunchKernelGGL(convert_kernel<P_F64>, g, b, 0, s, obs, N, D, Dp, V, rowbytes,
                           rowscale, vnorm2, nonfinite);
        break;
    case P_F32:
        hipLaunchKernelGGL(convert_kernel<P_F32>, g, b, 0, s, obs, N, D, Dp, V, rowbytes,
                           rowscale, vnorm2, nonfinite);
        break;
    case P_BF16X3:
        hipLaunchKernelGGL(convert_kernel<P_BF16X3>, g, b, 0, s, obs, N, D, Dp, V, rowbytes,
                           rowscale, vnorm2, nonfinite);
        break;
    case P_F16:
        hipLaunchKernelGGL(convert_kernel<P_F16>, g, b, 0, s, obs, N, D, Dp, V, rowbytes,
                           rowscale, vnorm2, nonfinite);
        break;
    case P_BF16:
        hipLaunchKernelGGL(convert_kernel<P_BF16>, g, b, 0, s, obs, N, D, Dp, V, rowbytes,
                           rowscale, vnorm2, nonfinite);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_colsum(const void *obs, int is_c128, int64_t N, int D, double *partials, int G,
                         hipStream_t s) {
    hipLaunchKernelGGL(colsum_kernel, dim3(G), dim3(512), 0, s, obs, is_c128, N, D, partials);
    return hipGetLastError();
}

hipError_t launch_sum(const double *x, int64_t n, double *partials, int G, double *out,
                      hipStream_t s) {
    hipLaunchKernelGGL(sum_kernel, dim3(G), dim3(256), 0, s, x, n, partials);
    hipLaunchKernelGGL(sum_kernel2, dim3(1), dim3(64), 0, s, partials, G, out);
    return hipGetLastError();
}

hipError_t launch_reduce(const double *partials, int G, int ncols, double *out, hipStream_t s) {
    hipLaunchKernelGGL(reduce_kernel, dim3((ncols + 63) / 64), dim3(512), 0, s, partials, G,
                       ncols, out);
    return hipGetLastError();
}

hipError_t launch_scale(const double *in, double *out, int n, double f, hipStream_t s) {
    hipLaunchKernelGGL(scale_kernel, dim3((n + 255) / 256), dim3(256), 0, s, in, out, n, f);
    return hipGetLastError();
}

hipError_t launch_logrho(const double *rho, float *l32, double *l64, int W, int Wp,
                         hipStream_t s) {
    hipLaunchKernelGGL(logrho_kernel, dim3(1), dim3(256), 0, s, rho, l32, l64, W, Wp);
    return hipGetLastError();
}

hipError_t launch_softmax(const double *eta, double *rho, float *l32, double *l64, int W, int Wp,
                          hipStream_t s) {
    hipLaunchKernelGGL(softmax_kernel, dim3(1), dim3(256), 0, s, eta, rho, l32, l64, W, Wp);
    return hipGetLastError();
}

hipError_t launch_template(const TplArgs &a, hipStream_t s) {
    const int64_t total = (int64_t)(a.Dp / 2) * a.Wp;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(template_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_reduce_finalize(const FinArgs &a, const double *partials, int G, int ncols,
                                  double *red, unsigned *count, hipStream_t s) {
    hipLaunchKernelGGL(reduce_finalize_kernel, dim3((ncols + kRedCols - 1) / kRedCols),
                       dim3(kFinThreads), 0, s, a, partials, G, ncols, red, count);
    return hipGetLastError();
}
hipError_t launch_histogram(const int32_t *err, int64_t n, int L, unsigned long long *counts,
                            hipStream_t s) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(histogram_kernel, dim3((unsigned)blocks), dim3(256),
                       (size_t)L * sizeof(unsigned int), s, err, n, L, counts);
    return hipGetLastError();
}

size_t pass_lds_bytes(int prec, int BM, int K, int Dp, int Wp, int LD) {
    return (size_t)pass_lds(prec, BM, K, Dp, Wp, LD ? 2 : 1).total;
}

typedef void (*pass_fn)(PassArgs);

// Events that time the next E+M pass launch of this host thread (the dispatch itself records
// them, so they bracket the kernel alone); null: untimed.
static thread_local hipEvent_t g_pass_ev[2] = {nullptr, nullptr};
void set_pass_events(hipEvent_t start, hipEvent_t stop) {
    g_pass_ev[0] = start;
    g_pass_ev[1] = stop;
}
static void launch_pass_fn(pass_fn f, int grid, size_t lds, hipStream_t s, const PassArgs &a) {
    if (g_pass_ev[0] || g_pass_ev[1])
        hipExtLaunchKernelGGL(f, dim3(grid), dim3(kThreads), (uint32_t)lds, s, g_pass_ev[0],
                              g_pass_ev[1], 0u, a);
    else
        hipLaunchKernelGGL(f, dim3(grid), dim3(kThreads), lds, s, a);
}

// General pass variants: (precision, rows per tile, waves along rows, loader).
#define SEM_PASS_VARIANTS(X)                                                                   \
    X(P_F64, 8, 1, 0) X(P_F64, 16, 1, 0) X(P_F64, 32, 1, 0) X(P_F64, 16, 1, 1)                 \
    X(P_F64, 32, 1, 1)                                                                         \
    X(P_F32, 16, 1, 0) X(P_F32, 32, 1, 0) X(P_F32, 32, 2, 0) X(P_F32, 64, 1, 0)                \
    X(P_F32, 64, 2, 0) X(P_F32, 64, 4, 0) X(P_F32, 16, 1, 1) X(P_F32, 32, 1, 1)                \
    X(P_F32, 32, 2, 1)                                                                         \
    X(P_BF16X3, 16, 1, 0) X(P_BF16X3, 32, 1, 0) X(P_BF16X3, 32, 2, 0) X(P_BF16X3, 64, 1, 0)     \
    X(P_BF16X3, 64, 2, 0) X(P_BF16X3, 64, 4, 0) X(P_BF16X3, 16, 1, 1)                          \
    X(P_F16, 16, 1, 0) X(P_F16, 32, 1, 0) X(P_F16, 32, 2, 0) X(P_F16, 64, 1, 0)                \
    X(P_F16, 64, 2, 0) X(P_F16, 64, 4, 0) X(P_F16, 16, 1, 1) X(P_F16, 32, 1, 1)                \
    X(P_F16, 32, 2, 1)                                                                         \
    X(P_BF16, 16, 1, 0) X(P_BF16, 32, 1, 0) X(P_BF16, 32, 2, 0) X(P_BF16, 64, 1, 0)            \
    X(P_BF16, 64, 2, 0) X(P_BF16, 64, 4, 0) X(P_BF16, 16, 1, 1) X(P_BF16, 32, 1, 1)            \
    X(P_BF16, 32, 2, 1)

static pass_fn find_pass(int prec, int BM, int WM, int LD) {
#define SEM_X(P, B, M, D)                                                                      \
    if (prec == P && BM == B && WM == M && LD == D) return pass_kernel<P, B, M, D>;
    SEM_PASS_VARIANTS(SEM_X)
#undef SEM_X
    return nullptr;
}

bool pass_variant_exists(int prec, int BM, int WM, int LD) {
    return find_pass(prec, BM, WM, LD) != nullptr;
}

static const char *kPrecName[] = {"f64", "f32", "bf16x3", "f16", "bf16"};

const char *pass_kernel_name(int prec, int BM, int WM, int LD) {
    static thread_local char buf[64];   // (per thread: callers copy it out)
    snprintf(buf, sizeof buf, "pass_kernel<%s,BM=%d,WM=%d,%s>", kPrecName[prec], BM, WM,
             LD ? "dma" : "reg");
    return buf;
}

hipError_t pass_setup(int prec, int BM, int WM, int LD, size_t lds, int *blocks_per_cu) {
    pass_fn f = find_pass(prec, BM, WM, LD);
    if (!f) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute((const void *)f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) (void)hipGetLastError();
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, (const void *)f, kThreads,
                                                        lds);
}

hipError_t launch_pass(int prec, int BM, int WM, int LD, const PassArgs &a, int grid, size_t lds,
                       hipStream_t s) {
    pass_fn f = find_pass(prec, BM, WM, LD);
    if (!f) return hipErrorInvalidValue;
    launch_pass_fn(f, grid, lds, s, a);
    return hipGetLastError();
}

// K-split variants: (precision, rows per tile, column tiles, k-steps per wave); Dp = 256 KSS.
#define SEM_KS_VARIANTS(X)                                                                     \
    X(P_BF16X3, 16, 4, 4) X(P_BF16X3, 16, 3, 4) X(P_F16, 16, 4, 4) X(P_F16, 16, 3, 4)           \
    X(P_BF16, 16, 4, 4) X(P_BF16, 16, 3, 4)

static pass_fn find_ks(int prec, int BM, int NT, int KSS, int QRY = 0) {
#define SEM_X(P, B, N, S)                                                                      \
    if (prec == P && BM == B && NT == N && KSS == S)                                           \
        return QRY ? pass_ks_kernel<P, B, N, S, 1> : pass_ks_kernel<P, B, N, S, 0>;
    SEM_KS_VARIANTS(SEM_X)
#undef SEM_X
    return nullptr;
}

bool ks_plan(int prec, int Dp, int Wp, int K, int *BM, int *NT, int *KSS) {
    const int nt = Wp / 16, kss = Dp / 256;
    if (Dp % 256 != 0 || 2 * K > 16 * (kThreads / 64)) return false;   // one U tile per wave
    // a_t and the phase rows are staged below the row factors at the start of a launch
    if (Dp / 2 > kStageA * kThreads || Wp * 2 * K > kStageE * kThreads) return false;
    for (int bm : {32, 16})
        if (find_ks(prec, bm, nt, kss) &&
            stage_a_e2_bytes(Dp / 2, Wp, K) <= ks_lds(prec, bm, nt, K, Dp, Wp).off_f) {
            *BM = bm;
            *NT = nt;
            *KSS = kss;
            return true;
        }
    return false;
}

size_t ks_lds_bytes(int prec, int BM, int NT, int K, int Dp, int Wp) {
    return (size_t)ks_lds(prec, BM, NT, K, Dp, Wp).total;
}

hipError_t launch_pass_ks(int prec, int BM, int NT, int KSS, const PassArgs &a, int grid,
                          size_t lds, hipStream_t s) {
    pass_fn f = find_ks(prec, BM, NT, KSS, (a.flags & PF_QUERY) ? 1 : 0);
    if (!f) return hipErrorInvalidValue;
    launch_pass_fn(f, grid, lds, s, a);
    return hipGetLastError();
}

hipError_t pass_ks_setup(int prec, int BM, int NT, int KSS, size_t lds, int *blocks_per_cu) {
    pass_fn f = find_ks(prec, BM, NT, KSS);
    if (!f) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute((const void *)f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) (void)hipGetLastError();
    e = hipFuncSetAttribute((const void *)find_ks(prec, BM, NT, KSS, 1),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) (void)hipGetLastError();
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, (const void *)f, kThreads,
                                                        lds);
}

const char *pass_ks_name(int prec, int BM, int NT, int KSS) {
    static thread_local char buf[64];   // (per thread: callers copy it out)
    snprintf(buf, sizeof buf, "pass_ks_kernel<%s,BM=%d,NT=%d,KSS=%d>", kPrecName[prec], BM, NT,
             KSS);
    return buf;
}

// Row-stream variants: (precision, window tiles).
#define SEM_KR_VARIANTS(X)                                                                     \
    X(P_F16, 1) X(P_F16, 2) X(P_F16, 3) X(P_F16, 4) X(P_BF16, 1) X(P_BF16, 2) X(P_BF16, 3)     \
    X(P_BF16, 4)

static pass_fn find_kr(int prec, int NT, int QRY = 0) {
#define SEM_X(P, N)                                                                            \
    if (prec == P && NT == N) return QRY ? pass_kr_kernel<P, N, 1> : pass_kr_kernel<P, N, 0>;
    SEM_KR_VARIANTS(SEM_X)
#undef SEM_X
    return nullptr;
}

bool kr_plan(int prec, int D, int Dp, int Q, int Wp, size_t lds_max, int *NT, size_t *lds) {
    if (prec != P_F16 && prec != P_BF16) return false;
    if (D != 512 || Dp != 1024) return false;
    if (Q != 8 && Q != 16 && Q != 32 && Q != 64) return false;
    const int nt = Wp / 16;
    if (nt < 1 || nt > 4 || !find_kr(prec, nt)) return false;
    const size_t l = (size_t)kr_lds(Dp).total;
    if (l > lds_max) return false;
    *NT = nt;
    *lds = l;
    return true;
}

hipError_t launch_pass_kr(int prec, int NT, const PassArgs &a, int grid, size_t lds,
                          hipStream_t s) {
    pass_fn f = find_kr(prec, NT, (a.flags & PF_QUERY) ? 1 : 0);
    if (!f) return hipErrorInvalidValue;
    launch_pass_fn(f, grid, lds, s, a);
    return hipGetLastError();
}

hipError_t pass_kr_setup(int prec, int NT, size_t lds, int *blocks_per_cu) {
    pass_fn f = find_kr(prec, NT);
    if (!f) return hipErrorInvalidValue;
    for (int q = 0; q < 2; ++q) {
        hipError_t e = hipFuncSetAttribute((const void *)find_kr(prec, NT, q),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) (void)hipGetLastError();
    }
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, (const void *)f, kThreads,
                                                        lds);
}

const char *pass_kr_name(int prec, int NT) {
    static thread_local char buf[64];   // (per thread: callers copy it out)
    snprintf(buf, sizeof buf, "pass_kr_kernel<%s,NT=%d>", kPrecName[prec], NT);
    return buf;
}

// Long-window FP32 GEMM-epilogue variants: (window tiles).
#define SEM_GM_VARIANTS(X)                                                                     \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)     \
    X(17) X(18) X(19) X(20) X(21) X(22) X(23) X(24)

static pass_fn find_gm(int NTC, int QRY = 0) {
#define SEM_X(N)                                                                               \
    if (NTC == N) return QRY ? pass_gm_kernel<N, 1> : pass_gm_kernel<N, 0>;
    SEM_GM_VARIANTS(SEM_X)
#undef SEM_X
    return nullptr;
}

bool gm_plan(int prec, int D, int K, int Q, int Wp, size_t lds_max, int *NTC, size_t *lds) {
    if (prec != P_F32 || D > 512 || Q % 8 != 0 || K > 32) return false;
    const int nt = Wp / 16;
    if (nt < 1 || nt > kGmMaxNT || !find_gm(nt)) return false;
    const size_t l = (size_t)gm_lds(nt, Wp, K, D).total;
    if (l > lds_max) return false;
    *NTC = nt;
    *lds = l;
    return true;
}

hipError_t launch_pass_gm(int NTC, const PassArgs &a, int grid, size_t lds, hipStream_t s) {
    pass_fn f = find_gm(NTC, (a.flags & PF_QUERY) ? 1 : 0);
    if (!f) return hipErrorInvalidValue;
    launch_pass_fn(f, grid, lds, s, a);
    return hipGetLastError();
}

hipError_t pass_gm_setup(int NTC, size_t lds, int *blocks_per_cu) {
    pass_fn f = find_gm(NTC);
    if (!f) return hipErrorInvalidValue;
    for (int q = 0; q < 2; ++q) {
        hipError_t e = hipFuncSetAttribute((const void *)find_gm(NTC, q),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) (void)hipGetLastError();
    }
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, (const void *)f, kThreads,
                                                        lds);
}

const char *pass_gm_name(int NTC) {
    static thread_local char buf[64];   // (per thread: callers copy it out)
    snprintf(buf, sizeof buf, "pass_gm_kernel<f32,BM=%d,NTC=%d>", kGmBM, NTC);
    return buf;
}

// Wide-row variants: (precision, window tiles per wave group, U chunk rows).
#define SEM_WIDE_VARIANTS(X)                                                                   \
    X(P_F16, 1, 32) X(P_F16, 2, 32) X(P_F16, 3, 32) X(P_F16, 4, 32)                             \
    X(P_BF16, 1, 32) X(P_BF16, 2, 32) X(P_BF16, 3, 32) X(P_BF16, 4, 32)

static pass_fn find_wide(int prec, int NTW, int UR) {
#define SEM_X(P, N, U)                                                                         \
    if (prec == P && NTW == N && UR == U) return pass_wide_kernel<P, N, U>;
    SEM_WIDE_VARIANTS(SEM_X)
#undef SEM_X
    return nullptr;
}

size_t wide_lds_bytes(int K, int Wp, int NTW, int UR) {
    return (size_t)wide_lds(K, Wp, NTW, UR).total;
}

bool wide_plan(int prec, int Wp, int K, size_t lds_max, int *NTW, int *UR) {
    const int ntw = (Wp / 16 + 3) / 4;
    const int ur = 32;
    if (!find_wide(prec, ntw, ur) || wide_lds_bytes(K, Wp, ntw, ur) > lds_max) return false;
    *NTW = ntw;
    *UR = ur;
    return true;
}

hipError_t launch_pass_wide(int prec, int NTW, int UR, const PassArgs &a, int grid, size_t lds,
                            hipStream_t s) {
    pass_fn f = find_wide(prec, NTW, UR);
    if (!f) return hipErrorInvalidValue;
    launch_pass_fn(f, grid, lds, s, a);
    return hipGetLastError();
}

hipError_t pass_wide_setup(int prec, int NTW, int UR, size_t lds, int *blocks_per_cu) {
    pass_fn f = find_wide(prec, NTW, UR);
    if (!f) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute((const void *)f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) (void)hipGetLastError();
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, (const void *)f, kThreads,
                                                        lds);
}

const char *pass_wide_name(int prec, int NTW, int UR) {
    static thread_local char buf[64];   // (per thread: callers copy it out)
    snprintf(buf, sizeof buf, "pass_wide_kernel<%s,BM=%d,NTW=%d,UR=%d>", kPrecName[prec],
             kWideBM, NTW, UR);
    return buf;
}

// Factored variants: (precision, window > 64, k-steps over [Re c | Im c]).
#define SEM_FAC_VARIANTS(X)                                                                    \
    X(P_F32, 0, 16, 8) X(P_F32, 1, 16, 8) X(P_F32, 0, 32, 8) X(P_F32, 1, 32, 8)                 \
    X(P_BF16X3, 0, 16, 8) X(P_BF16X3, 1, 16, 8) X(P_BF16X3, 0, 32, 8) X(P_BF16X3, 1, 32, 8)     \
    X(P_F16, 0, 16, 8) X(P_F16, 1, 16, 8) X(P_F16, 0, 32, 8) X(P_F16, 1, 32, 8)                 \
    X(P_BF16, 0, 16, 8) X(P_BF16, 1, 16, 8) X(P_BF16, 0, 32, 8) X(P_BF16, 1, 32, 8)             \
    X(P_F16, 1, 16, 16) X(P_F16, 1, 32, 16) X(P_BF16, 1, 16, 16) X(P_BF16, 1, 32, 16)

static pass_fn find_fac(int prec, int WIDE, int KCM, int EPL) {
#define SEM_X(P, Wd, KC, E)                                                                    \
    if (prec == P && WIDE == Wd && KCM == KC && EPL == E) return pass_fac_kernel<P, Wd, KC, E>;
    SEM_FAC_VARIANTS(SEM_X)
#undef SEM_X
    return nullptr;
}

bool fac_plan(int prec, int D, int Q, int K, int Wp, int gridL, size_t lds_max, int *WIDE,
              int *KCM, int *EPL, size_t *lds, int *BM) {
    int epl = 0;
    if (D == 512 && Q % 8 == 0) epl = 8;
    else if (D == 2048 && (prec == P_F16 || prec == P_BF16) && Q % 16 == 0) epl = 16;
    else return false;
    const int lpk = Q / epl;
    if (lpk & (lpk - 1)) return false;                       // lanes per frequency: 2^n
    const int kcm = 2 * K <= 64 ? 16 : (2 * K <= 128 ? 32 : 0);
    const int wide = (epl == 16 || Wp > 64) ? 1 : 0;
    if (!kcm || !find_fac(prec, wide, kcm, epl)) return false;
    const int bm = fac_bm(prec, epl);
    const int phl = (wide && gridL > 0 && gridL <= kFacPhLds) ? gridL : 0;
    const bool wbf = prec == P_BF16X3 && !wide && kcm == 16;
    const size_t b = (size_t)fac_lds(K, D, Wp, kcm, bm, epl, phl, wbf).total;
    if (b > lds_max) return false;
    *WIDE = wide;
    *KCM = kcm;
    *EPL = epl;
    *lds = b;
    *BM = bm;
    return true;
}

hipError_t launch_pass_fac(int prec, int WIDE, int KCM, int EPL, const PassArgs &a, int grid,
                           size_t lds, hipStream_t s) {
    pass_fn f = find_fac(prec, WIDE, KCM, EPL);
    if (!f) return hipErrorInvalidValue;
    launch_pass_fn(f, grid, lds, s, a);
    return hipGetLastError();
}

hipError_t pass_fac_setup(int prec, int WIDE, int KCM, int EPL, size_t lds, int *blocks_per_cu) {
    pass_fn f = find_fac(prec, WIDE, KCM, EPL);
    if (!f) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute((const void *)f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) (void)hipGetLastError();
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, (const void *)f, kThreads,
                                                        lds);
}

const char *pass_fac_name(int prec, int WIDE, int KCM, int EPL) {
    static thread_local char buf[64];   // (per thread: callers copy it out)
    snprintf(buf, sizeof buf, "pass_fac_kernel<%s,BM=%d,%s,KC=%d%s>", kPrecName[prec],
             fac_bm(prec, EPL), WIDE ? "L2" : "reg", KCM, EPL == 16 ? ",E16" : "");
    return buf;
}


// Symmetric-window factored pass variants: (precision, window tiles per wave, entries per lane).
#define SEM_FS_VARIANTS(X)                                                                     \
    X(P_F32, 1, 8) X(P_F32, 2, 8) X(P_BF16X3, 1, 8) X(P_BF16X3, 2, 8) X(P_F16, 1, 8)           \
    X(P_F16, 2, 8) X(P_BF16, 1, 8) X(P_BF16, 2, 8) X(P_F16, 1, 16) X(P_BF16, 1, 16)

static pass_fn find_fs(int prec, int MTW, int E) {
#define SEM_X(P, T, EE)                                                                        \
    if (prec == P && MTW == T && E == EE) return pass_fs_kernel<P, T, EE>;
    SEM_FS_VARIANTS(SEM_X)
#undef SEM_X
    return nullptr;
}

bool fs_plan(int prec, int D, int Q, int K, int L, int lo, int W, int Wp, bool grid,
             size_t lds_max, int *MTW, int *E, size_t *lds) {
    if (!grid || Wp <= 64) return false;
    int e = 0;
    if (D == 512 && Q % 8 == 0 && K <= 32) e = 8;
    else if (D == 2048 && (prec == P_F16 || prec == P_BF16) && Q % 16 == 0 && K <= 64) e = 16;
    else return false;
    const int lpk = Q / e;
    if (lpk & (lpk - 1)) return false;                       // lanes per frequency: 2^n
    if (W != L && !(W % 2 == 1 && fs_mod(lo + (W - 1) / 2, L) == 0))
        return false;                                        // not symmetric about offset 0
    const int MT = (fs_halves(L, lo, W) + 15) / 16;
    const int mtw = (MT + 7) / 8;
    if (!find_fs(prec, mtw, e)) return false;
    const size_t b = (size_t)(e == 8 ? fs_lds<8>(MT, D, Wp) : fs_lds<16>(MT, D, Wp)).total;
    if (b > lds_max) return false;
    *MTW = mtw;
    *E = e;
    *lds = b;
    return true;
}

hipError_t launch_pass_fs(int prec, int MTW, int E, const PassArgs &a, int grid, size_t lds,
                          hipStream_t s) {
    pass_fn f = find_fs(prec, MTW, E);
    if (!f) return hipErrorInvalidValue;
    launch_pass_fn(f, grid, lds, s, a);
    return hipGetLastError();
}

hipError_t pass_fs_setup(int prec, int MTW, int E, size_t lds, int *blocks_per_cu) {
    pass_fn f = find_fs(prec, MTW, E);
    if (!f) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute((const void *)f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) (void)hipGetLastError();
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, (const void *)f, kThreads,
                                                        lds);
}

const char *pass_fs_name(int prec, int MTW, int E) {
    static thread_local char buf[64];   // (per thread: callers copy it out)
    snprintf(buf, sizeof buf, "pass_fs_kernel<%s,BM=%d,MTW=%d%s>", kPrecName[prec],
             E == 16 ? 8 : 16, MTW, E == 16 ? ",E16" : "");
    return buf;
}

}  // namespace sem
