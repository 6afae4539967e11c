// HIP kernels of the Synch-EM iteration for gfx950 (CDNA4, wave64).
//
// One EM iteration (Algorithm "Synch-EM"; Section II-B eqs. (15), (17), (18); App. C eq. (42)):
//   template_kernel  T[:, i] = a_t o exp(-i kbar theta_{o_i}), written in MFMA B-fragment order
//   pass_kernel      per row tile: C = [Re V, Im V] [Re T; Im T] on matrix cores, then
//                    l_ji = 2 C_ji / sigma^2 + log rho_i, per-row log-sum-exp, posteriors,
//                    U_jk = sum_i w_ji exp(+i k theta_i), S_d += sum_j U_{j,kbar_d} v_jd,
//                    W_i += sum_j w_ji; FP64 per-workgroup partials
//   reduce_kernel    fixed-order FP64 sum of the partials
//   finalize_kernel  FP64: a_{t+1}, rho_{t+1}, log-likelihood, MAP objective, stopping metric
//
// The per-row constants -(||v_j||^2 + ||a||^2)/sigma^2 - D log(pi sigma^2) of the log-weights are
// left out of the pass (they cancel in the posteriors) and added back in FP64 in finalize_kernel.
#include "em_internal.h"

#include <math.h>
#include <stdio.h>

namespace sem {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
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
    for (int r = threadIdx.x; r < 2 * D; r += blockDim.x) {
        double s = 0.0;
        for (int64_t j = r0; j < r1; ++j) {
            s += is_c128 ? ((const double *)obs)[j * 2 * D + r]
                         : (double)((const float *)obs)[j * 2 * D + r];
        }
        partials[(int64_t)blockIdx.x * 2 * D + r] = s;
    }
}

// Fixed-order FP64 reduction over workgroup partials: out[c] = sum_b partials[b][c].
__global__ __launch_bounds__(512) void reduce_kernel(const double *partials, int G, int ncols,
                                                     double *out) {
    __shared__ double sh[8][64];
    const int cl = threadIdx.x & 63, gs = threadIdx.x >> 6;
    const int col = blockIdx.x * 64 + cl;
    double s = 0.0;
    if (col < ncols) {
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
            int64_t m = ((int64_t)k * (A.lo + i)) % A.L;
            if (m < 0) m += A.L;
            const double2 ph = A.phase[m];             // exp(+2 pi i m / L)
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

// LDS layout of the pass: [V tile: BM x RS bytes][C tile: BM x CSW][U chunk: UR x K][row factors]
constexpr int kUR = 16;                           // rows per U / M-step chunk
struct PassLds {
    int RS, CSW;
    int off_c, off_u, off_f, total;
};
__host__ __device__ inline PassLds pass_lds(int prec, int BM, int K, int Dp, int Wp) {
    PassLds l;
    const int rb = (int)row_bytes(prec, Dp);
    const int cs = prec == P_F64 ? 8 : 4;
    l.RS = rb + 16;
    l.CSW = Wp + 1;
    l.off_c = align_up(BM * l.RS, 16);
    l.off_u = align_up(l.off_c + BM * l.CSW * cs, 16);
    l.off_f = align_up(l.off_u + kUR * K * 2 * cs, 16);
    l.total = l.off_f + BM * 8 + 16;
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

// GEMM of one n-tile for MSW m-subtiles (rows ms*16 .. +15, ms = wm + m*WM), MFMA paths.
template <int P, int MSW, int WM>
__device__ __forceinline__ void gemm_ntile(f32x4 (&acc)[MSW], const uint8_t *Vs, int RS, int wm,
                                           int lane, int nt, int Dp, const void *Thi,
                                           const void *Tlo) {
    const int g = lane >> 4, rl = lane & 15;
#pragma unroll
    for (int m = 0; m < MSW; ++m) acc[m] = (f32x4){0.f, 0.f, 0.f, 0.f};
    if constexpr (P == P_F32) {
        const int KG = Dp / 16;
        const float4 *B = (const float4 *)Thi + (int64_t)nt * KG * 64 + lane;
        const uint8_t *Arow[MSW];
#pragma unroll
        for (int m = 0; m < MSW; ++m) Arow[m] = Vs + ((wm + m * WM) * 16 + rl) * RS + g * 16;
        float4 b = B[0];
#pragma unroll 2
        for (int kg = 0; kg < KG; ++kg) {
            const float4 bn = (kg + 1 < KG) ? B[(kg + 1) * 64] : b;
#pragma unroll
            for (int m = 0; m < MSW; ++m) {
                const float4 a = *(const float4 *)(Arow[m] + kg * 64);
                acc[m] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, acc[m], 0, 0, 0);
                acc[m] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, acc[m], 0, 0, 0);
                acc[m] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b.z, acc[m], 0, 0, 0);
                acc[m] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b.w, acc[m], 0, 0, 0);
            }
            b = bn;
        }
    } else {
        const int KS = Dp / 32;
        const uint4 *Bh = (const uint4 *)Thi + (int64_t)nt * KS * 64 + lane;
        const uint4 *Bl = (const uint4 *)Tlo + (int64_t)nt * KS * 64 + lane;
        const uint8_t *Arow[MSW];
#pragma unroll
        for (int m = 0; m < MSW; ++m) Arow[m] = Vs + ((wm + m * WM) * 16 + rl) * RS + g * 16;
        uint4 bh = Bh[0], bl = Bl[0];
#pragma unroll 2
        for (int ks = 0; ks < KS; ++ks) {
            uint4 bhn = bh, bln = bl;
            if (ks + 1 < KS) {
                bhn = Bh[(ks + 1) * 64];
                bln = Bl[(ks + 1) * 64];
            }
#pragma unroll
            for (int m = 0; m < MSW; ++m) {
                const uint4 ah = *(const uint4 *)(Arow[m] + ks * 64);
                if constexpr (P == P_F16) {
                    f16x8 A8 = __builtin_bit_cast(f16x8, ah);
                    acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                        A8, __builtin_bit_cast(f16x8, bl), acc[m], 0, 0, 0);
                    acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                        A8, __builtin_bit_cast(f16x8, bh), acc[m], 0, 0, 0);
                } else if constexpr (P == P_BF16) {
                    bf16x8 A8 = __builtin_bit_cast(bf16x8, ah);
                    acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        A8, __builtin_bit_cast(bf16x8, bl), acc[m], 0, 0, 0);
                    acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        A8, __builtin_bit_cast(bf16x8, bh), acc[m], 0, 0, 0);
                } else {  // P_BF16X3
                    const uint4 al = *(const uint4 *)(Arow[m] + 2 * Dp + ks * 64);
                    bf16x8 AH = __builtin_bit_cast(bf16x8, ah);
                    acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        AH, __builtin_bit_cast(bf16x8, bl), acc[m], 0, 0, 0);
                    acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        __builtin_bit_cast(bf16x8, al), __builtin_bit_cast(bf16x8, bh), acc[m],
                        0, 0, 0);
                    acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        AH, __builtin_bit_cast(bf16x8, bh), acc[m], 0, 0, 0);
                }
            }
            bh = bhn;
            bl = bln;
        }
    }
}

template <int P, int BM, int WM>
__global__ __launch_bounds__(kThreads) void pass_kernel(PassArgs A) {
    typedef typename PT<P>::CT CT;
    typedef typename PT<P>::CT2 CT2;
    constexpr int MS = BM / 16;
    constexpr int MSW = (MS / WM) > 0 ? MS / WM : 1;
    constexpr int TPR = kThreads / BM;            // threads per row in the row-wise phases
    constexpr int NPF = 16;                        // prefetch registers (16 B each) per thread

    if ((A.flags & PF_CHECK_STOP) && *A.stopped) return;

    extern __shared__ __align__(16) uint8_t smem[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const PassLds LY = pass_lds(P, BM, A.K, A.Dp, A.Wp);
    uint8_t *Vs = smem;
    CT *Cs = (CT *)(smem + LY.off_c);
    CT2 *Us = (CT2 *)(smem + LY.off_u);
    CT *rowf = (CT *)(smem + LY.off_f);

    const int64_t nrows_all = A.row_end - A.row_begin;
    const int64_t ntiles = (nrows_all + BM - 1) / BM;
    const int NT = A.Wp / 16;
    const int WN = 8 / WM;
    const int wn = wave % WN, wm = wave / WN;

    // Accumulators (FP64 across tiles).
    double2 accS[kMaxDPerThread];
    double accW[2];
    double acc_lse = 0.0, acc_wc = 0.0, acc_rows = 0.0;
#pragma unroll
    for (int c = 0; c < kMaxDPerThread; ++c) accS[c] = make_double2(0.0, 0.0);
    accW[0] = accW[1] = 0.0;

    const float tsc = (P == P_F64 || P == P_F32) ? 1.0f : *A.tscale;
    const bool accm = (A.flags & PF_ACC_M) != 0;

    // Register prefetch of the next tile: the tile is a contiguous byte range in HBM.
    u32x4 pf[NPF];
    auto issue_load = [&](int64_t tile) {
        const int64_t r0 = A.row_begin + tile * BM;
        const int64_t rows = (A.row_end - r0) < BM ? (A.row_end - r0) : BM;
        const int64_t nbytes = rows * A.rowbytes;
        const u32x4 *src = (const u32x4 *)(A.V + r0 * A.rowbytes);
#pragma unroll
        for (int c = 0; c < NPF; ++c) {
            const int64_t ch = (int64_t)c * kThreads + tid;
            pf[c] = (ch * 16 < nbytes) ? src[ch] : (u32x4){0u, 0u, 0u, 0u};
        }
    };
    auto store_tile = [&]() {
        const int64_t tbytes = (int64_t)BM * A.rowbytes;
#pragma unroll
        for (int c = 0; c < NPF; ++c) {
            const int64_t ch = (int64_t)c * kThreads + tid;
            if (ch * 16 < tbytes) {
                const int64_t byte = ch * 16;
                const int r = (int)(byte / A.rowbytes);
                const int off = (int)(byte - (int64_t)r * A.rowbytes);
                *(u32x4 *)(Vs + r * LY.RS + off) = pf[c];
            }
        }
    };

    int64_t tile = blockIdx.x;
    if (tile < ntiles) issue_load(tile);
    for (; tile < ntiles; tile += gridDim.x) {
        const int64_t r0 = A.row_begin + tile * BM;
        const int rows = (int)((A.row_end - r0) < BM ? (A.row_end - r0) : BM);
        __syncthreads();                                   // previous tile fully consumed
        store_tile();
        for (int j = tid; j < BM; j += kThreads) {
            CT f = (CT)A.coef;
            if (P != P_F64 && A.rowscale && j < rows) f *= (CT)A.rowscale[r0 + j] * (CT)tsc;
            rowf[j] = f;
        }
        __syncthreads();
        if (tile + gridDim.x < ntiles) issue_load(tile + gridDim.x);

        // ---- a3: correlations C and log-weights l' = coef * C + log rho  -> Cs
        if constexpr (P == P_F64) {
            const double *Td = (const double *)A.Thi;
            for (int o = tid; o < BM * A.Wp; o += kThreads) {
                const int r = o / A.Wp, col = o - r * A.Wp;
                const double *vr = (const double *)(Vs + r * LY.RS);
                double s = 0.0;
                for (int k = 0; k < A.Dp; ++k) s = fma(vr[k], Td[(int64_t)k * A.Wp + col], s);
                Cs[r * LY.CSW + col] = s * A.coef + A.logrho64[col];
            }
        } else {
            if (wm < WM) {
                for (int nt = wn; nt < NT; nt += WN) {
                    f32x4 acc[MSW];
                    gemm_ntile<P, MSW, WM>(acc, Vs, LY.RS, wm, lane, nt, A.Dp, A.Thi, A.Tlo);
                    const int col = nt * 16 + (lane & 15);
                    const float lr = A.logrho32[col];
#pragma unroll
                    for (int m = 0; m < MSW; ++m) {
                        const int rb = (wm + m * WM) * 16 + 4 * (lane >> 4);
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            Cs[(rb + q) * LY.CSW + col] = acc[m][q] * rowf[rb + q] + lr;
                    }
                }
            }
        }
        __syncthreads();

        // ---- a4: per-row log-sum-exp and posteriors (TPR threads per row)
        {
            const int r = tid / TPR, sub = tid % TPR;
            const bool valid = r < rows;
            CT *crow = Cs + r * LY.CSW;
            CT lse;
            if (A.flags & PF_LOAD_LSE) {
                lse = valid ? (CT)A.lse[r0 + r] : (CT)0;
            } else {
                CT m = -INFINITY;
                for (int i = sub; i < A.W; i += TPR) m = fmax(m, crow[i]);
                m = group_max(m, TPR);
                CT s = 0;
                for (int i = sub; i < A.W; i += TPR) s += exp(crow[i] - m);
                s = group_sum(s, TPR);
                lse = m + log(s);
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
                    w = exp(l - lse);
                    if (w > (CT)0) {
                        const CT lr = (P == P_F64) ? (CT)A.logrho64[i] : (CT)A.logrho32[i];
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
            wc = group_sum(wc, TPR);
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
                        const CT w1 = exp(b1 - lse), w2 = (A.W > 1) ? exp(b2 - lse) : (CT)0;
                        A.margin[qrow] = (float)(w1 - w2);
                    }
                }
            }
            if (sub == 0 && valid) {
                acc_lse += (double)lse;
                acc_wc += (double)wc / A.coef;            // sum_i w_ji C_ji
                acc_rows += 1.0;
                if (A.flags & PF_STORE_LSE) A.lse[r0 + r] = (double)lse;
            }
        }
        if (!accm) continue;
        __syncthreads();

        // ---- a5: W_t column sums, U = w E (scaled back to the observations' storage scale)
        for (int c = 0; c < 2; ++c) {
            const int i = tid + c * kThreads;
            if (i < A.Wp) {
                CT s = 0;
                for (int j = 0; j < rows; ++j) s += Cs[j * LY.CSW + i];
                accW[c] += (double)s;
            }
        }
        // U_jk = sum_i w_ji exp(+i k theta_i) for kUR rows at a time, then the M-step over them:
        // S_d += sum_j U_{j, kbar_d} v_jd (complex product, no conjugate).
        for (int j0 = 0; j0 < rows; j0 += kUR) {
            const int nr = (rows - j0) < kUR ? (rows - j0) : kUR;
            for (int p = tid; p < nr * A.K; p += kThreads) {
                const int jj = p / A.K, k = p - jj * A.K;
                const CT *wr = Cs + (j0 + jj) * LY.CSW;
                CT ur = 0, ui = 0;
                for (int i = 0; i < A.W; ++i) {
                    const CT w = wr[i];
                    if constexpr (P == P_F64) {
                        const double2 e = A.E64[i * A.K + k];
                        ur = fma(w, e.x, ur);
                        ui = fma(w, e.y, ui);
                    } else {
                        const float2 e = A.E32[i * A.K + k];
                        ur = fmaf(w, e.x, ur);
                        ui = fmaf(w, e.y, ui);
                    }
                }
                if (P != P_F64 && A.rowscale) {
                    const CT f = (CT)A.rowscale[r0 + j0 + jj];
                    ur *= f;
                    ui *= f;
                }
                CT2 u;
                u.x = ur;
                u.y = ui;
                Us[p] = u;
            }
            __syncthreads();
#pragma unroll
            for (int c = 0; c < kMaxDPerThread; ++c) {
                const int d = tid + c * kThreads;
                if (d < A.D) {
                    const int k = d / A.Q;
                    CT sr = 0, si = 0;
                    for (int jj = 0; jj < nr; ++jj) {
                        const CT2 v = load_v<P>(Vs + (j0 + jj) * LY.RS, d, A.Dp);
                        const CT2 u = Us[jj * A.K + k];
                        sr += u.x * v.x - u.y * v.y;
                        si += u.x * v.y + u.y * v.x;
                    }
                    accS[c].x += (double)sr;
                    accS[c].y += (double)si;
                }
            }
            __syncthreads();
        }
    }

    if (A.partials == nullptr) return;
    // ---- per-workgroup partials: S (2D), W (Wp), sum lse', sum w*C, rows
    double *Pp = A.partials + (int64_t)blockIdx.x * A.ncols;
    if (accm) {
#pragma unroll
        for (int c = 0; c < kMaxDPerThread; ++c) {
            const int d = tid + c * kThreads;
            if (d < A.D) {
                Pp[2 * d] = accS[c].x;
                Pp[2 * d + 1] = accS[c].y;
            }
        }
        for (int c = 0; c < 2; ++c) {
            const int i = tid + c * kThreads;
            if (i < A.Wp) Pp[2 * A.D + i] = accW[c];
        }
    } else {
        for (int i = tid; i < 2 * A.D + A.Wp; i += kThreads) Pp[i] = 0.0;
    }
    __syncthreads();
    double *sh = (double *)smem;
    const double s_lse = block_sum_d(acc_lse, sh, kThreads);
    const double s_wc = block_sum_d(acc_wc, sh, kThreads);
    const double s_rows = block_sum_d(acc_rows, sh, kThreads);
    if (tid == 0) {
        Pp[2 * A.D + A.Wp] = s_lse;
        Pp[2 * A.D + A.Wp + 1] = s_wc;
        Pp[2 * A.D + A.Wp + 2] = s_rows;
        Pp[2 * A.D + A.Wp + 3] = 0.0;
    }
}

// ------------------------------------------------------------------------------------------
// a6: FP64 finalize (one workgroup of 256).

__global__ __launch_bounds__(256) void finalize_kernel(FinArgs F) {
    if (F.mode == FIN_EM && *F.stopped) return;
    __shared__ double sh[256];
    __shared__ double2 anew[kMaxD];
    __shared__ double2 ck[kMaxK];
    const int t = threadIdx.x;
    const int D = F.D, W = F.W;
    const double N = (double)F.N;
    const double *S = F.red;
    const double *Wt = F.red + 2 * D;
    const double s_lse = F.red[2 * D + F.Wp];
    const double s_wc = F.red[2 * D + F.Wp + 1];

    double an2 = 0.0;
    for (int r = t; r < 2 * D; r += 256) an2 += F.a_in[r] * F.a_in[r];
    an2 = block_sum_d(an2, sh, 256);
    const double ll = s_lse - (F.sum_vn2 + N * an2) / F.sigma2 -
                      N * (double)D * log(M_PI * F.sigma2);

    if (F.mode == FIN_LL) {
        if (t == 0) F.out[0] = ll;
        return;
    }
    if (F.mode == FIN_GRAD) {
        const double c = F.g * 2.0 / F.sigma2;
        for (int r = t; r < 2 * D; r += 256) F.grad_a[r] = c * (S[r] - N * F.a_in[r]);
        if (F.grad_eta)
            for (int i = t; i < W; i += 256) F.grad_eta[i] = F.g * (Wt[i] - N * F.rho_in[i]);
        if (t == 0) {
            const double swr = F.sum_vn2 + N * an2 - 2.0 * s_wc;
            F.out[0] = ll;
            F.out[1] = F.g * (-N * (double)D / F.sigma2 + swr / (F.sigma2 * F.sigma2));
        }
        return;
    }

    // FIN_EM
    double jprior = 0.0;
    for (int i = t; i < W; i += 256)
        if (F.rho_bar[i] > 0.0 && F.gamma != 0.0) jprior += F.gamma * F.rho_bar[i] * log(F.rho_in[i]);
    for (int d = t; d < D; d += 256)
        if (F.gai) jprior -= F.gai[d] * (F.a_in[2 * d] * F.a_in[2 * d] + F.a_in[2 * d + 1] * F.a_in[2 * d + 1]);
    jprior = block_sum_d(jprior, sh, 256);

    double nn2 = 0.0, dl2 = 0.0;
    for (int d = t; d < D; d += 256) {
        const double den = N + (F.gai ? F.sigma2 * F.gai[d] : 0.0);
        const double2 an = make_double2(S[2 * d] / den, S[2 * d + 1] / den);
        anew[d] = an;
        nn2 += an.x * an.x + an.y * an.y;
        const double ex = an.x - F.a_in[2 * d], ey = an.y - F.a_in[2 * d + 1];
        dl2 += ex * ex + ey * ey;
    }
    nn2 = block_sum_d(nn2, sh, 256);
    dl2 = block_sum_d(dl2, sh, 256);
    // c_k = sum_q conj(a_new[k,q]) a_t[k,q]
    for (int k = t; k < F.K; k += 256) {
        double cr = 0.0, ci = 0.0;
        for (int q = 0; q < F.Q; ++q) {
            const int d = k * F.Q + q;
            const double2 an = anew[d];
            const double ar = F.a_in[2 * d], ai = F.a_in[2 * d + 1];
            cr += an.x * ar + an.y * ai;
            ci += an.x * ai - an.y * ar;
        }
        ck[k] = make_double2(cr, ci);
    }
    __syncthreads();
    // stopping metric min_l ||a_new - exp(-2 pi i kbar l / L) a_t||^2
    double best = INFINITY;
    for (int l = t; l < F.L; l += 256) {
        double re = 0.0;
        for (int k = 0; k < F.K; ++k) {
            const double2 ph = F.phase[((int64_t)k * l) % F.L];   // exp(+2 pi i k l / L)
            re += ck[k].x * ph.x + ck[k].y * ph.y;                 // Re(c_k exp(-2 pi i k l/L))
        }
        best = fmin(best, nn2 + an2 - 2.0 * re);
    }
    best = block_min_d(best, sh, 256);

    // rho update
    double tot = 0.0;
    for (int i = t; i < W; i += 256) tot += Wt[i] + F.gamma * F.rho_bar[i];
    tot = block_sum_d(tot, sh, 256);
    double ent = 0.0;
    for (int i = t; i < W; i += 256) {
        const double rn = F.update_rho ? (Wt[i] + F.gamma * F.rho_bar[i]) / tot : F.rho_in[i];
        if (rn > 0.0) ent -= rn * log(rn);
    }
    ent = block_sum_d(ent, sh, 256);
    __syncthreads();
    if (F.update_rho)
        for (int i = t; i < W; i += 256) F.rho[i] = (Wt[i] + F.gamma * F.rho_bar[i]) / tot;
    for (int d = t; d < D; d += 256) {
        F.a[2 * d] = anew[d].x;
        F.a[2 * d + 1] = anew[d].y;
    }
    __syncthreads();
    write_logrho(F.rho, F.logrho32, F.logrho64, W, F.Wp);
    if (t == 0) {
        const int64_t it = *F.t;
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

hipError_t launch_finalize(const FinArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(256), 0, s, a);
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

size_t pass_lds_bytes(int prec, int BM, int D, int K, int Dp, int Wp) {
    (void)D;
    return (size_t)pass_lds(prec, BM, K, Dp, Wp).total;
}

// Variant table: (precision, rows per tile, waves along rows).
#define SEM_PASS_VARIANTS(X)                                                                   \
    X(P_F64, 16, 1) X(P_F64, 32, 1) X(P_F64, 64, 1)                                            \
    X(P_F32, 16, 1) X(P_F32, 32, 1) X(P_F32, 32, 2) X(P_F32, 64, 1) X(P_F32, 64, 2)             \
    X(P_F32, 64, 4)                                                                            \
    X(P_BF16X3, 16, 1) X(P_BF16X3, 32, 1) X(P_BF16X3, 32, 2) X(P_BF16X3, 64, 1)                 \
    X(P_BF16X3, 64, 2) X(P_BF16X3, 64, 4)                                                      \
    X(P_F16, 16, 1) X(P_F16, 32, 1) X(P_F16, 32, 2) X(P_F16, 64, 1) X(P_F16, 64, 2)             \
    X(P_F16, 64, 4)                                                                            \
    X(P_BF16, 16, 1) X(P_BF16, 32, 1) X(P_BF16, 32, 2) X(P_BF16, 64, 1) X(P_BF16, 64, 2)        \
    X(P_BF16, 64, 4)

typedef void (*pass_fn)(PassArgs);

static pass_fn find_pass(int prec, int BM, int WM) {
#define SEM_X(P, B, M)                                                                         \
    if (prec == P && BM == B && WM == M) return pass_kernel<P, B, M>;
    SEM_PASS_VARIANTS(SEM_X)
#undef SEM_X
    return nullptr;
}

bool pass_variant_exists(int prec, int BM, int WM) { return find_pass(prec, BM, WM) != nullptr; }

const char *pass_kernel_name(int prec, int BM, int WM) {
    static char buf[64];
    static const char *pn[] = {"f64", "f32", "bf16x3", "f16", "bf16"};
    snprintf(buf, sizeof buf, "pass_kernel<%s,BM=%d,WM=%d>", pn[prec], BM, WM);
    return buf;
}

hipError_t pass_set_lds_limit(int prec, int BM, int WM, size_t lds) {
    pass_fn f = find_pass(prec, BM, WM);
    if (!f) return hipErrorInvalidValue;
    return hipFuncSetAttribute((const void *)f, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds);
}

hipError_t pass_occupancy(int prec, int BM, int WM, size_t lds, int *blocks_per_cu) {
    pass_fn f = find_pass(prec, BM, WM);
    if (!f) return hipErrorInvalidValue;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, (const void *)f, kThreads,
                                                        lds);
}

hipError_t launch_pass(int prec, int BM, int WM, const PassArgs &a, int grid, size_t lds,
                       hipStream_t s) {
    pass_fn f = find_pass(prec, BM, WM);
    if (!f) return hipErrorInvalidValue;
    hipLaunchKernelGGL(f, dim3(grid), dim3(kThreads), lds, s, a);
    return hipGetLastError();
}

}  // namespace sem
