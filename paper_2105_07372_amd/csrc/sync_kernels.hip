// HIP kernels of Synchronize and Match for gfx950 (CDNA4, wave64): the step before the EM path
// (§II-A "Angular synchronization", §III-A Algorithm "Synchronize and Match").
//
//   relrot_kernel   relative rotation of every pair of the subset S_P: the per-frequency sums
//                   c_ijk = sum_q conj(v_ikq) v_jkq, then f_ij(l) = Re sum_k c_ijk exp(-i k 2 pi
//                   l / L) for all L grid rotations on FP32 matrix cores, its argmax (the rotation
//                   that best maps v_j onto v_i) and the gap to the runner-up
//   ppm_kernel      one projected power iteration z <- phase(H z), H_ij = exp(+i 2 pi rel_ij / L),
//                   in FP64
//   nearest_kernel  for each observation the nearest member of S_P (squared distance without
//                   rotation, ||v_n||^2 - 2 Re <v_i, v_n>, on FP32 matrix cores), the member itself
//                   excluded, with the gap to the runner-up (nearest_lds_kernel: rows up to 1024
//                   reals staged in LDS, 32 per workgroup)
//   gather / align  theta_i = phi_{nn_i}; v_i o exp(+i kbar theta_i)
//
// Ties in an argmax or argmin go to the lowest index.
#include "em_internal.h"

#include <math.h>

#include <mutex>

namespace sem {

typedef float f32x4s __attribute__((ext_vector_type(4)));

// The best value, its index and the runner-up value of a set; merge() is order-independent:
// the best is the largest value (lowest index among equals), the runner-up the largest of the
// rest.
struct Top2 {
    float b;
    int i;
    float s;
};
__device__ __forceinline__ Top2 top2_merge(Top2 A, Top2 B) {
    if (B.b > A.b || (B.b == A.b && B.i < A.i)) return Top2{B.b, B.i, fmaxf(A.b, B.s)};
    return Top2{A.b, A.i, fmaxf(A.s, B.b)};
}
__device__ __forceinline__ Top2 top2_shfl_xor(Top2 t, int m) {
    return Top2{__shfl_xor(t.b, m), __shfl_xor(t.i, m), __shfl_xor(t.s, m)};
}

constexpr int kSyncThreads = 256;

// Grid (ceil(P / 16), P): workgroup (jt, i) handles the pairs (i, 16 jt .. 16 jt + 15).
// B: Lp x K2 floats, row l = [cos(k 2 pi l / L) (k < K) | sin(k 2 pi l / L) (k < K) | 0 ..],
// zero rows for l >= L.  K2 = 2K rounded up to a multiple of 4.
__global__ __launch_bounds__(kSyncThreads) void relrot_kernel(const float2 *V, int P, int K, int Q,
                                                              int L, int Lp, int K2,
                                                              const float *B, int *rel,
                                                              float *gap, float *dot0) {
    extern __shared__ __align__(16) uint8_t smem[];
    const int D = K * Q;
    const int CBW = K2 + 4;
    float2 *vi = (float2 *)smem;                           // D entries of v_i
    float *cs = (float *)(smem + ((D * 8 + 15) / 16) * 16); // 16 x CBW: [Re c | Im c | 0]
    Top2 *red = (Top2 *)(cs + 16 * CBW);                   // 4 waves x 16 rows
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int i = blockIdx.y, j0 = blockIdx.x * 16;
    for (int d = t; d < D; d += kSyncThreads) vi[d] = V[(int64_t)i * D + d];
    __syncthreads();
    // c for the 16 pairs: thread (p, s) sums the frequencies k = s, s + 16, ...
    {
        const int p = t >> 4, s = t & 15, j = j0 + p;
        for (int k = s; k < K2; k += 16) {
            float v = 0.f;
            if (j < P && k < 2 * K) {
                const int kk = k < K ? k : k - K;
                float cr = 0.f, ci = 0.f;
                const float2 *vj = V + (int64_t)j * D + kk * Q;
                for (int q = 0; q < Q; ++q) {
                    const float2 a = vi[kk * Q + q], b = vj[q];
                    cr += a.x * b.x + a.y * b.y;               // Re conj(v_i) v_j
                    ci += a.x * b.y - a.y * b.x;               // Im conj(v_i) v_j
                }
                v = k < K ? cr : ci;
            }
            cs[p * CBW + k] = v;
        }
    }
    __syncthreads();
    // f (16 pairs x Lp) = [Re c | Im c] . B^T on FP32 matrix cores; wave w takes column tiles
    // w, w + 4, ...; lane (g, c) holds rows 4 g .. 4 g + 3 of column 16 n + c
    const int g = lane >> 4, c = lane & 15;
    Top2 best[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) best[q] = Top2{-INFINITY, 0x7fffffff, -INFINITY};
    const int NTc = Lp / 16;
    for (int n = wave; n < NTc; n += kSyncThreads / 64) {
        f32x4s acc = (f32x4s){0.f, 0.f, 0.f, 0.f};
        const float *bb = B + (int64_t)(16 * n + c) * K2;
        for (int kk = 0; kk < K2 / 4; ++kk) {
            const float a = cs[c * CBW + 4 * kk + g];
            const float b = bb[4 * kk + g];
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
        }
        const int l = 16 * n + c;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (l < L) best[q] = top2_merge(best[q], Top2{acc[q], l, -INFINITY});
            if (l == 0) {
                const int j = j0 + 4 * g + q;
                if (j < P) dot0[(int64_t)i * P + j] = acc[q];
            }
        }
    }
    // the 16 lanes of a row group, then the four waves in order
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int m = 1; m < 16; m <<= 1) best[q] = top2_merge(best[q], top2_shfl_xor(best[q], m));
    if (c == 0)
#pragma unroll
        for (int q = 0; q < 4; ++q) red[wave * 16 + 4 * g + q] = best[q];
    __syncthreads();
    if (t < 16) {
        Top2 r = red[t];
        for (int w = 1; w < kSyncThreads / 64; ++w) r = top2_merge(r, red[w * 16 + t]);
        const int j = j0 + t;
        if (j < P) {
            rel[(int64_t)i * P + j] = r.i;
            gap[(int64_t)i * P + j] = r.b - r.s;
        }
    }
}

// The same estimate for a 16 x 16 tile of pairs (i in 16 it .., j in 16 jt ..) with both
// contractions on FP32 matrix cores, for 2K <= 64 and Lp <= 384.
//  1. c_ijk for the 256 pairs: per frequency k (wave w takes k = w, w + 4, ..) two real products
//     over the 2Q interleaved reals of frequency k: Re c = [a_r a_i] . [b_r b_i] and
//     Im c = [a_r a_i] . [b_i -b_r]; lane group g loads reals 16 s + 4 g .. + 3 of its i row (A)
//     and j row (B) as one 16-byte read and feeds four MFMA k-steps (2Q a multiple of 16).
//  2. f (256 pairs x Lp) = [Re c | Im c] . B^T: wave w owns the column tiles w, w + 4, .. (NW of
//     them), their B fragments in registers for the whole workgroup; per 16-pair row tile m the
//     A fragments come from LDS once and serve all the wave's column tiles; the top-2 of each
//     pair is merged over the 16 lanes of a row group, then over the waves through LDS.
template <int NW>
__global__ __launch_bounds__(kSyncThreads) void relrot_tile_kernel(const float2 *V, int P, int K,
                                                                   int Q, int L, int Lp,
                                                                   const float *B, int *rel,
                                                                   float *gap, float *dot0) {
    constexpr int KK = 16, K2 = 64, CBW = K2 + 4;
    __shared__ float cs[256 * CBW];
    __shared__ Top2 red[4 * 256];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int g = lane >> 4, c = lane & 15;
    const int i0 = blockIdx.y * 16, j0 = blockIdx.x * 16;
    const int D = K * Q;
    // ---- 1. per-frequency sums on matrix cores
    for (int col = t; col < 256 * CBW; col += kSyncThreads) cs[col] = 0.f;
    __syncthreads();
    {
        const int ia = i0 + c < P ? i0 + c : P - 1, jb = j0 + c < P ? j0 + c : P - 1;
        const int NC = 2 * Q / 16;
        for (int k = wave; k < K; k += 4) {
            const float4 *pa = (const float4 *)(V + (int64_t)ia * D + k * Q);
            const float4 *pb = (const float4 *)(V + (int64_t)jb * D + k * Q);
            f32x4s cr = (f32x4s){0.f, 0.f, 0.f, 0.f}, ci = cr;
            for (int sc = 0; sc < NC; ++sc) {
                const float4 a = pa[4 * sc + g], b = pb[4 * sc + g];
                // reals (x, y) and (z, w) are (re, im) pairs: [b_i, -b_r] per pair for Im
                cr = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, cr, 0, 0, 0);
                cr = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, cr, 0, 0, 0);
                cr = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b.z, cr, 0, 0, 0);
                cr = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b.w, cr, 0, 0, 0);
                ci = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.y, ci, 0, 0, 0);
                ci = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, -b.x, ci, 0, 0, 0);
                ci = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b.w, ci, 0, 0, 0);
                ci = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, -b.z, ci, 0, 0, 0);
            }
            // cr[q] = Re c for i = i0 + 4 g + q, j = j0 + c
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int pr = (4 * g + q) * 16 + c;
                cs[pr * CBW + k] = cr[q];
                cs[pr * CBW + K + k] = ci[q];
            }
        }
    }
    __syncthreads();
    // ---- 2. the L-grid correlations and their top-2
    float bf[NW][KK];
#pragma unroll
    for (int u = 0; u < NW; ++u) {
        const int n = wave + 4 * u;
        const bool ok = 16 * n < Lp;
        const float *bb = B + (int64_t)(ok ? 16 * n + c : 0) * K2;
#pragma unroll
        for (int kk = 0; kk < KK; ++kk) bf[u][kk] = ok ? bb[4 * kk + g] : 0.f;
    }
    for (int m = 0; m < 16; ++m) {
        float af[KK];
#pragma unroll
        for (int kk = 0; kk < KK; ++kk) af[kk] = cs[(16 * m + c) * CBW + 4 * kk + g];
        Top2 best[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) best[q] = Top2{-INFINITY, 0x7fffffff, -INFINITY};
#pragma unroll
        for (int u = 0; u < NW; ++u) {
            const int n = wave + 4 * u;
            if (16 * n >= Lp) break;
            f32x4s acc = (f32x4s){0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kk = 0; kk < KK; ++kk)
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(af[kk], bf[u][kk], acc, 0, 0, 0);
            const int l = 16 * n + c;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (l < L) best[q] = top2_merge(best[q], Top2{acc[q], l, -INFINITY});
                if (l == 0) {
                    // pair (16 m + 4 g + q): i = i0 + (16 m + 4 g + q) / 16, j = j0 + .. % 16
                    const int pr = 16 * m + 4 * g + q, ii = i0 + pr / 16, jj = j0 + pr % 16;
                    if (ii < P && jj < P) dot0[(int64_t)ii * P + jj] = acc[q];
                }
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int mm = 1; mm < 16; mm <<= 1)
                best[q] = top2_merge(best[q], top2_shfl_xor(best[q], mm));
        if (c == 0)
#pragma unroll
            for (int q = 0; q < 4; ++q) red[wave * 256 + 16 * m + 4 * g + q] = best[q];
    }
    __syncthreads();
    {
        Top2 r = red[t];
        for (int w = 1; w < 4; ++w) r = top2_merge(r, red[w * 256 + t]);
        const int ii = i0 + t / 16, jj = j0 + t % 16;
        if (ii < P && jj < P) {
            rel[(int64_t)ii * P + jj] = r.i;
            gap[(int64_t)ii * P + jj] = r.b - r.s;
        }
    }
}

// One projected power iteration: 4 rows per workgroup, 64 lanes per row summing j = lane,
// lane + 64, .. in FP64, then a butterfly over the wave; z_out = y / |y| (z_in kept if y = 0).
// PHL: the L phases are first copied to LDS (L <= kPpmPhLds), so the per-entry lookups are LDS
// reads rather than scattered global ones.
constexpr int kPpmPhLds = 2048;
template <bool PHL>
__global__ __launch_bounds__(kSyncThreads) void ppm_kernel(const int *rel, int P, int L,
                                                           const double2 *ph,
                                                           const double2 *z_in,
                                                           double2 *z_out) {
    __shared__ double2 phs[PHL ? kPpmPhLds : 1];
    if constexpr (PHL) {
        for (int m = threadIdx.x; m < L; m += kSyncThreads) phs[m] = ph[m];
        __syncthreads();
    }
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= P) return;                                     // whole waves leave together
    double yr = 0.0, yi = 0.0;
#pragma unroll 4
    for (int j = lane; j < P; j += 64) {
        int m = rel[(int64_t)i * P + j];
        if (m < 0 || m >= L) {                              // (reduced mod L)
            m %= L;
            if (m < 0) m += L;
        }
        double2 h;
        if constexpr (PHL) h = phs[m]; else h = ph[m];
        const double2 z = z_in[j];
        yr += h.x * z.x - h.y * z.y;
        yi += h.x * z.y + h.y * z.x;
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        yr += __shfl_xor(yr, m);
        yi += __shfl_xor(yi, m);
    }
    if (lane == 0) {
        const double a = sqrt(yr * yr + yi * yi);
        z_out[i] = a > 0.0 ? make_double2(yr / a, yi / a) : z_in[i];
    }
}

__global__ void angle_kernel(const double2 *z, int P, double *theta) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < P) theta[i] = atan2(z[i].y, z[i].x);
}

__global__ void ones_kernel(double2 *z, int P) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < P) z[i] = make_double2(1.0, 0.0);
}

// ||v_n||^2 of the first P rows (FP64 sum, stored as float).
__global__ void rownorm_kernel(const float2 *V, int64_t P, int D, float *nrm) {
    const int64_t n = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (n >= P) return;
    double s = 0.0;
    for (int d = lane; d < D; d += 64) {
        const float2 v = V[n * D + d];
        s += (double)v.x * v.x + (double)v.y * v.y;
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m);
    if (lane == 0) nrm[n] = (float)s;
}

// Nearest member of S_P for 16 observations per workgroup: wave w takes the reference tiles
// w, w + 4, ..; the contraction over the 2D reals runs in chunks of 16, lane group g loading the
// four consecutive reals 16 s + 4 g .. + 3 of its row (query) and column (reference) as one
// 16-byte read and feeding them to four MFMA k-steps (the same permutation of k on both sides).
// Requires 2D % 16 == 0.
__global__ __launch_bounds__(kSyncThreads) void nearest_kernel(const float2 *V, int64_t N,
                                                               int64_t P, int D,
                                                               const float *nrm, int *nn,
                                                               float *gap) {
    __shared__ Top2 red[4 * 16];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int g = lane >> 4, c = lane & 15;
    const int64_t r0 = (int64_t)blockIdx.x * 16;
    const int64_t qrow = r0 + c < N ? r0 + c : N - 1;
    const float4 *qa = (const float4 *)(V + qrow * D);
    const int NC = 2 * D / 16;                             // chunks of 16 reals
    Top2 best[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) best[q] = Top2{-INFINITY, 0x7fffffff, -INFINITY};
    const int64_t NTr = (P + 15) / 16;
    for (int64_t n = wave; n < NTr; n += kSyncThreads / 64) {
        const int64_t ref = 16 * n + c;
        const float4 *rb = (const float4 *)(V + (ref < P ? ref : P - 1) * D);
        f32x4s acc = (f32x4s){0.f, 0.f, 0.f, 0.f};
        for (int s = 0; s < NC; ++s) {
            const float4 a = qa[4 * s + g], b = rb[4 * s + g];
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b.z, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b.w, acc, 0, 0, 0);
        }
        // acc[q] = Re <v_row, v_ref> for row r0 + 4 g + q, reference 16 n + c
        if (ref < P) {
            const float nr = nrm[ref];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t row = r0 + 4 * g + q;
                if (row != ref)                              // a member never matches itself
                    best[q] = top2_merge(best[q], Top2{2.f * acc[q] - nr, (int)ref, -INFINITY});
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int m = 1; m < 16; m <<= 1) best[q] = top2_merge(best[q], top2_shfl_xor(best[q], m));
    if (c == 0)
#pragma unroll
        for (int q = 0; q < 4; ++q) red[wave * 16 + 4 * g + q] = best[q];
    __syncthreads();
    if (t < 16) {
        Top2 r = red[t];
        for (int w = 1; w < kSyncThreads / 64; ++w) r = top2_merge(r, red[w * 16 + t]);
        const int64_t row = r0 + t;
        if (row < N) {
            nn[row] = r.i;
            gap[row] = r.b - r.s;                           // in squared-distance units
        }
    }
}

// The same search for 32 observations per workgroup of 512 threads, their rows staged once in
// LDS (rows padded by 4 floats so that the 16 lanes of a row group read distinct banks): wave w
// takes the reference tiles w, w + 8, ..; each 16-byte reference load serves the four MFMA
// k-steps of both 16-row halves.  For 2D <= 1024 and 2D % 16 == 0.
constexpr int kNnThreads = 512;
__global__ __launch_bounds__(kNnThreads) void nearest_lds_kernel(const float2 *V, int64_t N,
                                                                 int64_t P, int D,
                                                                 const float *nrm, int *nn,
                                                                 float *gap) {
    extern __shared__ __align__(16) uint8_t smem[];
    const int RS = 2 * D + 4;                               // floats per staged row
    float *Aq = (float *)smem;
    Top2 *red = (Top2 *)(Aq + 32 * RS);                     // 8 waves x 32 rows
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int g = lane >> 4, c = lane & 15;
    const int64_t r0 = (int64_t)blockIdx.x * 32;
    const int F4 = 2 * D / 4;                               // float4 per row
    for (int q = t; q < 32 * F4; q += kNnThreads) {
        const int r = q / F4, f = q - r * F4;
        const int64_t row = r0 + r < N ? r0 + r : N - 1;
        *(float4 *)(Aq + r * RS + 4 * f) = ((const float4 *)(V + row * D))[f];
    }
    __syncthreads();
    const int NC = 2 * D / 16;
    Top2 best[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) best[q] = Top2{-INFINITY, 0x7fffffff, -INFINITY};
    const int64_t NTr = (P + 15) / 16;
    const float *a0p = Aq + c * RS + 4 * g, *a1p = Aq + (16 + c) * RS + 4 * g;
    for (int64_t n = wave; n < NTr; n += kNnThreads / 64) {
        const int64_t ref = 16 * n + c;
        const float4 *rb = (const float4 *)(V + (ref < P ? ref : P - 1) * D);
        f32x4s acc0 = (f32x4s){0.f, 0.f, 0.f, 0.f}, acc1 = acc0;
        for (int sc = 0; sc < NC; ++sc) {
            const float4 b = rb[4 * sc + g];
            const float4 a0 = *(const float4 *)(a0p + 16 * sc);
            const float4 a1 = *(const float4 *)(a1p + 16 * sc);
            acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0.x, b.x, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1.x, b.x, acc1, 0, 0, 0);
            acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0.y, b.y, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1.y, b.y, acc1, 0, 0, 0);
            acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0.z, b.z, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1.z, b.z, acc1, 0, 0, 0);
            acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0.w, b.w, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1.w, b.w, acc1, 0, 0, 0);
        }
        if (ref < P) {
            const float nr = nrm[ref];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (r0 + 4 * g + q != ref)
                    best[q] = top2_merge(best[q], Top2{2.f * acc0[q] - nr, (int)ref, -INFINITY});
                if (r0 + 16 + 4 * g + q != ref)
                    best[4 + q] =
                        top2_merge(best[4 + q], Top2{2.f * acc1[q] - nr, (int)ref, -INFINITY});
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
        for (int m = 1; m < 16; m <<= 1) best[q] = top2_merge(best[q], top2_shfl_xor(best[q], m));
    if (c == 0)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            red[wave * 32 + 4 * g + q] = best[q];
            red[wave * 32 + 16 + 4 * g + q] = best[4 + q];
        }
    __syncthreads();
    if (t < 32) {
        Top2 r = red[t];
        for (int w = 1; w < kNnThreads / 64; ++w) r = top2_merge(r, red[w * 32 + t]);
        const int64_t row = r0 + t;
        if (row < N) {
            nn[row] = r.i;
            gap[row] = r.b - r.s;
        }
    }
}

// (an index outside [0, P), left by non-finite distances, gives NaN instead of a read)
__global__ void gather_kernel(const double *phi, int64_t P, const int *nn, int64_t N,
                              double *theta) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) {
        const int n = nn[i];
        theta[i] = (n >= 0 && n < P) ? phi[n] : NAN;
    }
}

// out[i][d] = v[i][d] exp(+i kbar_d theta_i): one thread per (row, frequency), FP64 phase.
__global__ void align_kernel(const float2 *V, int64_t N, int K, int Q, const double *theta,
                             float2 *out) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N * K) return;
    const int64_t i = p / K;
    const int k = (int)(p - i * K);
    double sn, cn;
    sincos((double)k * theta[i], &sn, &cn);
    const int64_t base = i * (int64_t)K * Q + (int64_t)k * Q;
    for (int q = 0; q < Q; ++q) {
        const float2 v = V[base + q];
        out[base + q] = make_float2((float)(v.x * cn - v.y * sn), (float)(v.x * sn + v.y * cn));
    }
}

// Column sums of the aligned observations: workgroup b sums rows b, b + G, .. of
// v_i o exp(+i kbar theta_i) for its columns in FP64 (phase in FP64); partials [G][2D].
__global__ __launch_bounds__(256) void aligned_colsum_kernel(const float2 *V, int64_t N, int K,
                                                             int Q, const double *theta,
                                                             double *partials) {
    const int D = K * Q;
    for (int d = threadIdx.x; d < D; d += 256) {
        const int k = d / Q;
        double sr = 0.0, si = 0.0;
        for (int64_t i = blockIdx.x; i < N; i += gridDim.x) {
            double sn, cn;
            sincos((double)k * theta[i], &sn, &cn);
            const float2 v = V[i * D + d];
            sr += v.x * cn - v.y * sn;
            si += v.x * sn + v.y * cn;
        }
        partials[(int64_t)blockIdx.x * 2 * D + 2 * d] = sr;
        partials[(int64_t)blockIdx.x * 2 * D + 2 * d + 1] = si;
    }
}

// floor((theta_hat - theta - 2 pi lc / L) L / (2 pi)) mod L, in FP64.
__global__ void error_bins_kernel(const double *theta_hat, const double *theta, int64_t N, int L,
                                  int lc, int *bins) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double e = theta_hat[i] - theta[i] - 2.0 * M_PI * lc / L;
    const double f = floor(e * L / (2.0 * M_PI));
    int64_t b = (int64_t)fmod(f, (double)L);
    if (b < 0) b += L;
    bins[i] = (int)b;
}

// ------------------------------------------------------------------------------------------
// launchers

size_t relrot_lds_bytes(int K, int Q) {
    const int D = K * Q, K2 = (2 * K + 3) / 4 * 4;
    return (size_t)((D * 8 + 15) / 16) * 16 + (size_t)16 * (K2 + 4) * 4 + 64 * sizeof(Top2);
}

bool relrot_tiled(int K, int Q, int L) {
    const int Lp = (L + 15) / 16 * 16;
    return (2 * K + 3) / 4 * 4 <= 64 && (2 * Q) % 16 == 0 && Lp <= 16 * 4 * 6;
}

hipError_t launch_relrot(const float2 *V, int P, int K, int Q, int L, const float *B, int *rel,
                         float *gap, float *dot0, hipStream_t s) {
    const int Lp = (L + 15) / 16 * 16, K2 = (2 * K + 3) / 4 * 4;
    if (relrot_tiled(K, Q, L)) {
        // B is laid out with row stride 64 for this kernel (see em_relative_rotations)
        const int NT = Lp / 16, NW = (NT + 3) / 4;
        const dim3 grid((P + 15) / 16, (P + 15) / 16);
#define SEM_RT(W)                                                                                  case W:                                                                                            hipLaunchKernelGGL(relrot_tile_kernel<W>, grid, dim3(kSyncThreads), 0, s, V, P, K, Q, L,                            Lp, B, rel, gap, dot0);                                                     break;
        switch (NW) {
            SEM_RT(1) SEM_RT(2) SEM_RT(3) SEM_RT(4) SEM_RT(5) SEM_RT(6)
        default: return hipErrorInvalidValue;
        }
#undef SEM_RT
        return hipGetLastError();
    }
    const size_t lds = relrot_lds_bytes(K, Q);
    hipError_t e = hipFuncSetAttribute((const void *)relrot_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) (void)hipGetLastError();
    hipLaunchKernelGGL(relrot_kernel, dim3((P + 15) / 16, P), dim3(kSyncThreads), lds, s, V, P,
                       K, Q, L, Lp, K2, B, rel, gap, dot0);
    return hipGetLastError();
}

hipError_t launch_ppm(const int *rel, int P, int L, const double2 *ph, double2 *z0, double2 *z1,
                      int iters, double *theta, hipStream_t s) {
    hipLaunchKernelGGL(ones_kernel, dim3((P + 255) / 256), dim3(256), 0, s, z0, P);
    for (int it = 0; it < iters; ++it) {
        if (L <= kPpmPhLds)
            hipLaunchKernelGGL(ppm_kernel<true>, dim3((P + 3) / 4), dim3(kSyncThreads), 0, s, rel,
                               P, L, ph, (it & 1) ? z1 : z0, (it & 1) ? z0 : z1);
        else
            hipLaunchKernelGGL(ppm_kernel<false>, dim3((P + 3) / 4), dim3(kSyncThreads), 0, s,
                               rel, P, L, ph, (it & 1) ? z1 : z0, (it & 1) ? z0 : z1);
    }
    hipLaunchKernelGGL(angle_kernel, dim3((P + 255) / 256), dim3(256), 0, s,
                       (iters & 1) ? z1 : z0, P, theta);
    return hipGetLastError();
}

hipError_t launch_nearest(const float2 *V, int64_t N, int64_t P, int D, float *nrm, int *nn,
                          float *gap, hipStream_t s) {
    hipLaunchKernelGGL(rownorm_kernel, dim3((unsigned)((P + 3) / 4)), dim3(256), 0, s, V, P, D,
                       nrm);
    if (2 * D <= 1024 && (2 * D) % 16 == 0) {
        const size_t lds = (size_t)32 * (2 * D + 4) * 4 + (size_t)8 * 32 * sizeof(Top2);
        hipError_t e = hipFuncSetAttribute((const void *)nearest_lds_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) (void)hipGetLastError();
        hipLaunchKernelGGL(nearest_lds_kernel, dim3((unsigned)((N + 31) / 32)), dim3(kNnThreads),
                           lds, s, V, N, P, D, nrm, nn, gap);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(nearest_kernel, dim3((unsigned)((N + 15) / 16)), dim3(kSyncThreads), 0, s,
                       V, N, P, D, nrm, nn, gap);
    return hipGetLastError();
}

hipError_t launch_gather(const double *phi, int64_t P, const int *nn, int64_t N, double *theta,
                         hipStream_t s) {
    hipLaunchKernelGGL(gather_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, phi, P,
                       nn, N, theta);
    return hipGetLastError();
}

hipError_t launch_align(const float2 *V, int64_t N, int K, int Q, const double *theta,
                        float2 *out, hipStream_t s) {
    const int64_t total = N * K;
    hipLaunchKernelGGL(align_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, V, N,
                       K, Q, theta, out);
    return hipGetLastError();
}

hipError_t launch_aligned_colsum(const float2 *V, int64_t N, int K, int Q, const double *theta,
                                double *partials, int G, hipStream_t s) {
    hipLaunchKernelGGL(aligned_colsum_kernel, dim3(G), dim3(256), 0, s, V, N, K, Q, theta,
                       partials);
    return hipGetLastError();
}

// Scratch of the aligned-mean entry point that allocates nothing: the per-workgroup partial
// column sums, kAlignedMeanBlocks x 2 kMaxD doubles (8 MiB), one copy per device for the life of
// the process.  Host code never passes the array's name to a kernel (on the host it is only a
// stand-in for the symbol); it passes the device address that hipGetSymbolAddress returns for
// the current device, looked up once per device and kept.
static __device__ __align__(256) double scratch[(size_t)kAlignedMeanBlocks * 2 * kMaxD];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch(double **ptr, size_t *bytes) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = (double *)p;
    }
    *ptr = g_scratch_ptr[dev];
    *bytes = sizeof(scratch);
    return hipSuccess;
}

hipError_t launch_error_bins(const double *theta_hat, const double *theta, int64_t N, int L,
                             int lc, int *bins, hipStream_t s) {
    hipLaunchKernelGGL(error_bins_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s,
                       theta_hat, theta, N, L, lc, bins);
    return hipGetLastError();
}

}  // namespace sem
