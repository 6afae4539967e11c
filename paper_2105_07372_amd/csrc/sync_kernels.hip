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
//                   excluded, with the gap to the runner-up
//   gather / align  theta_i = phi_{nn_i}; v_i o exp(+i kbar theta_i)
//
// Ties in an argmax or argmin go to the lowest index.
#include "em_internal.h"

#include <math.h>

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

// One projected power iteration: 4 rows per workgroup, 64 lanes per row summing j = lane,
// lane + 64, .. in FP64, then a butterfly over the wave; z_out = y / |y| (z_in kept if y = 0).
__global__ __launch_bounds__(kSyncThreads) void ppm_kernel(const int *rel, int P, int L,
                                                           const double2 *ph,
                                                           const double2 *z_in,
                                                           double2 *z_out) {
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= P) return;                                     // whole waves leave together
    double yr = 0.0, yi = 0.0;
    for (int j = lane; j < P; j += 64) {
        int m = rel[(int64_t)i * P + j] % L;
        if (m < 0) m += L;
        const double2 h = ph[m], z = z_in[j];
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

hipError_t launch_relrot(const float2 *V, int P, int K, int Q, int L, const float *B, int *rel,
                         float *gap, float *dot0, hipStream_t s) {
    const int Lp = (L + 15) / 16 * 16, K2 = (2 * K + 3) / 4 * 4;
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
        hipLaunchKernelGGL(ppm_kernel, dim3((P + 3) / 4), dim3(kSyncThreads), 0, s, rel, P, L,
                           ph, (it & 1) ? z1 : z0, (it & 1) ? z0 : z1);
    }
    hipLaunchKernelGGL(angle_kernel, dim3((P + 255) / 256), dim3(256), 0, s,
                       (iters & 1) ? z1 : z0, P, theta);
    return hipGetLastError();
}

hipError_t launch_nearest(const float2 *V, int64_t N, int64_t P, int D, float *nrm, int *nn,
                          float *gap, hipStream_t s) {
    hipLaunchKernelGGL(rownorm_kernel, dim3((unsigned)((P + 3) / 4)), dim3(256), 0, s, V, P, D,
                       nrm);
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

hipError_t launch_error_bins(const double *theta_hat, const double *theta, int64_t N, int L,
                             int lc, int *bins, hipStream_t s) {
    hipLaunchKernelGGL(error_bins_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s,
                       theta_hat, theta, N, L, lc, bins);
    return hipGetLastError();
}

}  // namespace sem
