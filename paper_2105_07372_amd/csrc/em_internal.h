// Internal interface between the host library (em_api.cpp) and the HIP kernels (em_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sem {

enum Prec : int { P_F64 = 0, P_F32 = 1, P_BF16X3 = 2, P_F16 = 3, P_BF16 = 4 };

// What one E(+M) pass does.
enum PassFlags : int {
    PF_ACC_M = 1,       // accumulate the M-step sums S, W_t and sum w*C into per-block partials
    PF_STORE_LSE = 2,   // write the per-row log-sum-exp (checkpoint)
    PF_LOAD_LSE = 4,    // normalise with the stored per-row log-sum-exp (adjoint recompute)
    PF_QUERY = 8,       // write posterior rows, argmax and margin
    PF_CHECK_STOP = 16  // return at once when the context's stop flag is set
};

enum FinMode : int { FIN_EM = 0, FIN_LL = 1, FIN_GRAD = 2 };

constexpr int kThreads = 512;        // threads per workgroup of the E+M pass (8 wave64)
constexpr int kMaxDPerThread = 4;    // D <= 4 * kThreads
constexpr int kMaxD = kMaxDPerThread * kThreads;
constexpr int kMaxSyncP = 8192;      // Synchronize and Match: subset size
constexpr int kMaxSyncL = 4096;      // ... and rotation grid
constexpr int kMaxWp = 1024;         // padded window <= 2 * kThreads
constexpr int kMaxK = 512;
constexpr int kStatsCap = 1024;
constexpr int kWideBM = 128;         // rows per tile of the wide-row pass
constexpr int kRegTileChunks = 8;    // register-staged tiles: <= 8 x 16 B per thread (64 KiB)

// Bytes of one stored observation row (all planes), Dp reals wide.
__host__ __device__ inline int64_t row_bytes(int prec, int Dp) {
    switch (prec) {
    case P_F64: return (int64_t)Dp * 8;
    case P_F32: return (int64_t)Dp * 4;
    case P_BF16X3: return (int64_t)Dp * 4;      // bf16 hi plane then bf16 lo plane
    default: return (int64_t)Dp * 2;            // fp16 or bf16, one plane
    }
}

struct PassArgs {
    const double *a;           // 2D: the coefficients (the K-split pass builds its template)
    const uint8_t *V;          // N rows of rowbytes
    int64_t rowbytes;
    const float *rowscale;     // per-row factor undoing the storage scaling (null: 1)
    const void *Thi, *Tlo;     // template, MFMA B-fragment order (see template_kernel)
    const float *tscale;       // device scalar: factor undoing the template scaling
    const float *logrho32;     // Wp, -inf on padding and on zero entries
    const double *logrho64;
    const float *E2;           // Wp x 2K: [Re exp(+i k theta_i) | Im ...] (zero rows on padding)
    const double2 *E64;        // Wp x K: exp(+i k theta_i), FP64 path
    const double2 *phase;      // L: exp(+2 pi i m / L) (grid windows: E[i, k] = phase[k o_i mod L])
    int L, lo, grid;           // grid: the window is the offsets lo .. lo + W - 1 (no angle list)
    int64_t row_begin, row_end;
    int D, K, Q, Dp, W, Wp;
    double coef;               // 2 / sigma^2
    int flags;
    double *partials;          // [gridDim.x][ncols]
    int ncols;
    double *lse;               // per absolute row
    float *post;               // (row - row_begin) x W
    int32_t *argmax;
    float *margin;
    const int *stopped;
};

struct FinArgs {
    int mode;
    const double *red;         // reduced partials: S[2D], W[Wp], sum lse', sum w*C, rows
    int64_t N;
    int D, K, Q, W, Wp, L;
    double sigma2, gamma, tol, g;
    int update_rho;
    double sum_vn2;            // sum_j ||v_j||^2 (FP64, from the unrounded observations)
    const double *rho_bar;     // W
    const double *gai;         // D or null
    const double2 *phase;      // L: exp(+2 pi i m / L)
    const double *a_in;        // 2D: the coefficients the pass used
    const double *rho_in;      // W: the distribution the pass used
    // FIN_EM: state update
    double *a, *rho;
    int64_t *t;
    int *stopped;
    double *ll_last;
    double *stats;
    float *logrho32;
    double *logrho64;
    // FIN_LL / FIN_GRAD outputs
    double *out;               // [0] = log-likelihood, [1] = g * dLL/dsigma2
    double *grad_a;            // 2D
    double *grad_eta;          // W
};

struct TplArgs {
    const double *a;
    int D, K, Q, Dp, W, Wp, prec;
    const double2 *E64;        // Wp x K: exp(+i k theta_i)
    void *Thi, *Tlo;
    float *tscale;
    const int *stopped;
};

// Launchers (em_kernels.hip).  All return hipSuccess or the launch error.
hipError_t launch_convert(int prec, const void *obs, int64_t N, int D, int Dp, uint8_t *V,
                          int64_t rowbytes, float *rowscale, double *vnorm2, int *nonfinite,
                          hipStream_t s);
hipError_t launch_colsum(const void *obs, int is_c128, int64_t N, int D, double *partials,
                         int G, hipStream_t s);
hipError_t launch_reduce(const double *partials, int G, int ncols, double *out, hipStream_t s);
// Fixed-order FP64 sum of n values: G workgroup partials (partials holds G doubles), then out.
hipError_t launch_sum(const double *x, int64_t n, double *partials, int G, double *out,
                      hipStream_t s);
hipError_t launch_scale(const double *in, double *out, int n, double factor, hipStream_t s);
hipError_t launch_template(const TplArgs &a, hipStream_t s);
hipError_t launch_pass(int prec, int BM, int WM, int LD, const PassArgs &a, int grid, size_t lds,
                       hipStream_t s);
// Events for the next E+M pass launch of the calling thread (recorded by the dispatch, so they
// time the kernel alone); (null, null) turns it off.  Every launch_pass* honours them.
void set_pass_events(hipEvent_t start, hipEvent_t stop);
// The fixed-order sum of G rows of ncols partials into red, then the finalize on red (F.red must
// be red), in one launch.  count: one device counter per context, 0 before the first launch and
// left at 0 by every launch; launches that share it must not overlap.
hipError_t launch_reduce_finalize(const FinArgs &a, const double *partials, int G, int ncols,
                                  double *red, unsigned *count, hipStream_t s);
// Synchronize and Match (sync_kernels.hip).  B: Lp x K2 floats of cos | sin (see relrot_kernel).
// true when the 16 x 16 pair-tile kernel serves (2K <= 64, Q % 8 == 0, L <= 384); its cos | sin
// table then has row stride 64, else 2K rounded up to 4
bool relrot_tiled(int K, int Q, int L);
hipError_t launch_relrot(const float2 *V, int P, int K, int Q, int L, const float *B, int *rel,
                         float *gap, float *dot0, hipStream_t s);
hipError_t launch_ppm(const int *rel, int P, int L, const double2 *ph, double2 *z0, double2 *z1,
                      int iters, double *theta, hipStream_t s);
hipError_t launch_nearest(const float2 *V, int64_t N, int64_t P, int D, float *nrm, int *nn,
                          float *gap, hipStream_t s);
hipError_t launch_gather(const double *phi, int64_t P, const int *nn, int64_t N, double *theta,
                         hipStream_t s);
hipError_t launch_align(const float2 *V, int64_t N, int K, int Q, const double *theta,
                        float2 *out, hipStream_t s);
hipError_t launch_aligned_colsum(const float2 *V, int64_t N, int K, int Q, const double *theta,
                                double *partials, int G, hipStream_t s);
hipError_t launch_error_bins(const double *theta_hat, const double *theta, int64_t N, int L,
                             int lc, int *bins, hipStream_t s);
// Workgroups of the aligned column sums (both aligned-mean entry points use this many, so their
// fixed-order sums are the same).
constexpr int kAlignedMeanBlocks = 256;
// The library's own device scratch for em_aligned_mean_noalloc (sync_kernels.hip): the current
// device's address of a static array of kAlignedMeanBlocks x 2 kMaxD doubles, looked up once per
// device (*bytes receives its size).
hipError_t noalloc_scratch(double **ptr, size_t *bytes);
hipError_t launch_softmax(const double *eta, double *rho, float *logrho32, double *logrho64,
                          int W, int Wp, hipStream_t s);
hipError_t launch_logrho(const double *rho, float *logrho32, double *logrho64, int W, int Wp,
                         hipStream_t s);
hipError_t launch_histogram(const int32_t *err, int64_t n, int L, unsigned long long *counts,
                            hipStream_t s);
size_t pass_lds_bytes(int prec, int BM, int K, int Dp, int Wp, int LD);
hipError_t pass_setup(int prec, int BM, int WM, int LD, size_t lds, int *blocks_per_cu);
const char *pass_kernel_name(int prec, int BM, int WM, int LD);
bool pass_variant_exists(int prec, int BM, int WM, int LD);
bool ks_plan(int prec, int Dp, int Wp, int K, int *BM, int *NT, int *KSS);
size_t ks_lds_bytes(int prec, int BM, int NT, int K, int Dp, int Wp);
hipError_t launch_pass_ks(int prec, int BM, int NT, int KSS, const PassArgs &a, int grid,
                          size_t lds, hipStream_t s);
hipError_t pass_ks_setup(int prec, int BM, int NT, int KSS, size_t lds, int *blocks_per_cu);
const char *pass_ks_name(int prec, int BM, int NT, int KSS);
// Row-stream correlation pass (one 16-bit plane, D = 512, Q in {8, 16, 32, 64}, Wp <= 64).
bool kr_plan(int prec, int D, int Dp, int Q, int Wp, size_t lds_max, int *NT, size_t *lds);
hipError_t launch_pass_kr(int prec, int NT, const PassArgs &a, int grid, size_t lds,
                          hipStream_t s);
hipError_t pass_kr_setup(int prec, int NT, size_t lds, int *blocks_per_cu);
const char *pass_kr_name(int prec, int NT);
// Long-window FP32 pass built as a GEMM with the posterior and M-step as epilogue (D <= 512,
// Q % 8 == 0, K <= 32, Wp <= 384).
bool gm_plan(int prec, int D, int K, int Q, int Wp, size_t lds_max, int *NTC, size_t *lds);
hipError_t launch_pass_gm(int NTC, const PassArgs &a, int grid, size_t lds, hipStream_t s);
hipError_t pass_gm_setup(int NTC, size_t lds, int *blocks_per_cu);
const char *pass_gm_name(int NTC);
bool wide_plan(int prec, int Wp, int K, size_t lds_max, int *NTW, int *UR);
size_t wide_lds_bytes(int K, int Wp, int NTW, int UR);
hipError_t launch_pass_wide(int prec, int NTW, int UR, const PassArgs &a, int grid, size_t lds,
                            hipStream_t s);
hipError_t pass_wide_setup(int prec, int NTW, int UR, size_t lds, int *blocks_per_cu);
const char *pass_wide_name(int prec, int NTW, int UR);
// gridL: L for a grid window (its phase table may be staged in LDS), 0 for an angle list
bool fac_plan(int prec, int D, int Q, int K, int Wp, int gridL, size_t lds_max, int *WIDE,
              int *KCM, int *EPL, size_t *lds, int *BM);
hipError_t launch_pass_fac(int prec, int WIDE, int KCM, int EPL, const PassArgs &a, int grid,
                           size_t lds, hipStream_t s);
hipError_t pass_fac_setup(int prec, int WIDE, int KCM, int EPL, size_t lds, int *blocks_per_cu);
const char *pass_fac_name(int prec, int WIDE, int KCM, int EPL);
// The factored pass over a window symmetric about offset 0 (W = L, or lo = -h with W = 2h + 1),
// on the grid with Wp > 64: D = 512 (K <= 32; E = 8 entries per lane) or D = 2048 in one 16-bit
// plane (K <= 64; E = 16, rows over wave pairs); EM and log-likelihood passes only (no posterior
// queries, no stored or loaded per-row log-sum-exps).  MTW: window tiles of 16 per wave.
bool fs_plan(int prec, int D, int Q, int K, int L, int lo, int W, int Wp, bool grid,
             size_t lds_max, int *MTW, int *E, size_t *lds);
hipError_t launch_pass_fs(int prec, int MTW, int E, const PassArgs &a, int grid, size_t lds,
                          hipStream_t s);
hipError_t pass_fs_setup(int prec, int MTW, int E, size_t lds, int *blocks_per_cu);
const char *pass_fs_name(int prec, int MTW, int E);

}  // namespace sem
