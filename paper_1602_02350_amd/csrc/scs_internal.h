// Internal declarations shared by the HIP sources of libscs (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "scs.h"

namespace scs {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);

struct Status {
  int code = SCS_OK;
};

#define SCS_HIP(call)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) {                                                            \
      ::scs::set_error(std::string(#call) + ": " + hipGetErrorString(e_));             \
      return SCS_EDEVICE;                                                              \
    }                                                                                  \
  } while (0)

#define SCS_CHECK(expr)          \
  do {                           \
    int rc_ = (expr);            \
    if (rc_ < 0) return rc_;     \
  } while (0)

// ---------------------------------------------------------------- device helpers
__device__ __forceinline__ float warp_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ __forceinline__ double warp_sum_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Sum over the 64 lanes with DPP row rotations (by 8, 4, 2, 1 inside each 16-lane row) and the
// gfx950 row swaps (16-lane rows 0<->1, 2<->3, then the 32-lane halves): a few cycles per step
// instead of an LDS round trip per step. Every lane ends with a sum of all 64 values; lanes may
// differ in the last bit (their summation orders differ), so use one lane's value.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double swap_add_d(double v, bool halves) {
  const long long b = __double_as_longlong(v);
  const unsigned int lo = (unsigned int)b, hi = (unsigned int)(b >> 32);
  if (halves) {
    auto pl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    auto ph = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    return __longlong_as_double(((long long)ph[0] << 32) | pl[0]) + __longlong_as_double(((long long)ph[1] << 32) | pl[1]);
  }
  auto pl = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  auto ph = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  return __longlong_as_double(((long long)ph[0] << 32) | pl[0]) + __longlong_as_double(((long long)ph[1] << 32) | pl[1]);
}
__device__ __forceinline__ double wave_sum_d_fast(double v) {
  v += dpp_d<0x128>(v);
  v += dpp_d<0x124>(v);
  v += dpp_d<0x122>(v);
  v += dpp_d<0x121>(v);
  v = swap_add_d(v, false);
  return swap_add_d(v, true);
}

__device__ __forceinline__ double warp_max_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// FP32 -> BF16 with round-to-nearest-even (NaN kept quiet).
// FP32 -> BF16 with round-to-nearest-even (gfx950 converts in hardware, v_cvt_pk_bf16_f32).
typedef __bf16 bf16x2_v __attribute__((ext_vector_type(2)));
typedef float f32x2_v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint16_t f32_to_bf16(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
// two values in one word, the first in the low half
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
  const f32x2_v v = {lo, hi};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_v));
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011): 10 rounds of the 4x32 bijection,
// multipliers 0xD2511F53 / 0xCD9E8D57, key bumped by the Weyl constants between rounds.
struct U4 {
  uint32_t x, y, z, w;
};
__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    U4 n;
    n.x = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
    n.y = (uint32_t)p1;
    n.z = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
    n.w = (uint32_t)p0;
    c = n;
  }
  return c;
}

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Problem owning unit x of a flattened batched grid: the largest p with prefix[p] <= x.
__device__ __forceinline__ int find_prob(const int64_t* prefix, int nprob, int64_t x) {
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------- device-side solver state
// One record per problem, written by the kernels and read back by the host at the end.
struct SolveState {
  int done;          // 1 once the stop rule holds or an error was found: later kernels return at once
  int status;        // SCS_* outcome
  int epochs;        // epochs whose inner loop ran
  int k_used;
  double obj;        // L at the last evaluated snapshot
  double obj0;       // L at the first snapshot (divergence reference)
  double gnorm2;     // ||grad L~||^2 at the last evaluated snapshot
  double cert;
  double beta_sum;   // sum_i ||a_i||^2 over the n + d rows
  double eta;
  double s;          // sqrt(lam_k + lambda) (1 if k = 0)
  double lam_top;
  double wsum;       // total quantized sampling weight (as double, for reporting)
  int backoffs;      // step-size halvings after rejected snapshots (eta is scaled by 2^-backoffs)
  int pad_i;
  double pad[2];
};
constexpr int kMaxBackoffs = 6;  // a further rejected snapshot ends the solve with SCS_DIVERGED

// The decision on an evaluated snapshot (one thread; obj = L at the snapshot, gn = ||mu||^2 with
// mu = grad L~ = P^{-1/2} grad L). Returns 0 = continue, 1 = stop (converged), 2 = diverged (restore,
// stop), 3 = non-finite input, 4 = rejected snapshot (restore the previous one, halve the step size
// and continue), and records the outcome in the state.
// Certificate: H~ = P^{-1/2} H P^{-1/2} >= lambda P^{-1} >= lambda / (lam_1 + lambda) I, so
// L - L* <= ||mu||^2 / (2 lambda_min(H~)) <= ||mu||^2 (lam_1 + lambda) / (2 lambda); with P = I the
// factor lam_1 + lambda is 1.
__device__ __forceinline__ int snapshot_decision(SolveState* state, double obj, double gn, const double* lam, int k,
                                                 double lambda, int first, int stop_rule, double eps,
                                                 double f_star) {
  const double lam_top = k > 0 ? fmax(lam[0], 0.0) : 0.0;
  const double cert = gn * (k > 0 ? lam_top + lambda : 1.0) / (2.0 * lambda);
  const bool finite = isfinite(obj) && isfinite(gn);
  int action = 0;
  if (first) {
    if (!finite) action = 3;
    else state->obj0 = obj;
  } else if (!finite || obj > 10.0 * state->obj0) {
    if (state->backoffs < kMaxBackoffs) {
      state->backoffs += 1;
      action = 4;
    } else {
      action = 2;
    }
  }
  if (action == 0) {
    state->obj = obj;
    state->gnorm2 = gn;
    state->cert = cert;
    if (stop_rule == SCS_STOP_CERTIFICATE && cert <= eps) action = 1;
    if (stop_rule == SCS_STOP_GAP && obj - f_star <= eps) action = 1;
  }
  if (action == 1) {
    state->done = 1;
    state->status = SCS_OK;
  } else if (action == 2) {
    state->done = 1;
    state->status = SCS_DIVERGED;
  } else if (action == 3) {
    state->done = 1;
    state->status = SCS_ENONFINITE;
  }
  return action;
}

// ---------------------------------------------------------------- launchers (defined in the .hip files)
// rng
int launch_gaussian(hipStream_t st, uint64_t seed, int64_t count, float* out);
// uniform != 0: q_i = 1/N for every component instead of q_i proportional to beta_i
int launch_sampler_prepare(hipStream_t st, const float* beta, int64_t N, uint64_t* cum, double* scratch,
                           int64_t scratch_len, SolveState* state, int uniform = 0);
int launch_sample(hipStream_t st, const uint64_t* cum, int64_t N, int64_t n_rows, uint64_t seed, int epoch,
                  int64_t per_epoch, int64_t count, int32_t* idx, float* scale, const SolveState* state);
int launch_index_scale(hipStream_t st, const uint64_t* cum, int64_t N, int64_t n_rows, const int32_t* idx,
                       int64_t count, float* scale, const SolveState* state);
// the same from FP64 beta, and with the scales 1/(n q_i) kept in FP64 (the FP64 path)
int launch_sampler_prepare(hipStream_t st, const double* beta, int64_t N, uint64_t* cum, double* scratch,
                           int64_t scratch_len, SolveState* state, int uniform = 0);
int launch_sample(hipStream_t st, const uint64_t* cum, int64_t N, int64_t n_rows, uint64_t seed, int epoch,
                  int64_t per_epoch, int64_t count, int32_t* idx, double* scale, const SolveState* state);
int launch_index_scale(hipStream_t st, const uint64_t* cum, int64_t N, int64_t n_rows, const int32_t* idx,
                       int64_t count, double* scale, const SolveState* state);
int64_t sampler_scratch_len(int64_t N);

// gemm (MFMA)
// A launch gated on a device counter does nothing once *count >= total (read at kernel entry): the
// shared-X gradient GEMMs of a regularization path skip epochs in which every solve has stopped.
struct Gate {
  const int* count = nullptr;
  int total = 0;
};
// pad16: also store columns N .. (N rounded up to 16) - 1, which come out zero
int launch_gemm_nt_longk(hipStream_t st, int bf16, const float* A, int64_t M, int64_t K, int64_t lda,
                         const float* Bt, int64_t N, int64_t ldb, float* C, int64_t ldc, bool pad16 = false,
                         Gate gate = Gate());
// Leading dimension (and zero-padded width) the wide GEMM wants for operands with K columns.
int gemm_wide_kpad(int64_t K);
// Rows the wide GEMM reads from Bt: N rounded up to 64.
inline int64_t gemm_wide_bt_rows(int64_t N) { return (N + 63) / 64 * 64; }
int launch_gemm_nt_wide(hipStream_t st, int bf16, const float* A, int64_t M, int64_t K, int64_t lda,
                        const float* Bt, int64_t N, int64_t ldb, float alpha, const float* C0, int64_t ldc0,
                        float beta, const double* beta_dev, float diag, const double* diag_dev, int out_bf16,
                        void* C, int64_t ldc, float* rownorm2);
// Row chunks for gemm_tn_splitk over R rows (the same operands as the launch that follows).
int64_t gemm_tn_splitk_chunks(int64_t R, int64_t M, int64_t N, const float* A, int64_t lda, const float* B,
                              int64_t ldb);
// Partial Gram matrices W^T W of row chunks of W (R x L, leading dimension ldw, L <= 64) in FP32 MFMA:
// partial[c][i L + j] for the gram_rr_f32_parts(R) chunks c
int64_t gram_rr_f32_parts(int64_t R);
int launch_gram_rr_f32(hipStream_t st, const float* W, int64_t R, int L, int64_t ldw, float* partial);
int launch_gemm_tn_splitk(hipStream_t st, int bf16, const float* A, int64_t R, int64_t M, int64_t lda,
                          const float* B, int64_t N, int64_t ldb, float* partial, int64_t chunk_rows,
                          int64_t nchunks, Gate gate = Gate());
int launch_reduce_partials_f64(hipStream_t st, const float* partial, int64_t nchunks, int64_t elems,
                               double scale, double* out);
// fp64 dense
int launch_gemm64(hipStream_t st, int64_t M, int64_t N, int64_t K, const double* A, int64_t a_rs,
                  int64_t a_cs, const double* B, int64_t b_rs, int64_t b_cs, double* C, int64_t ldc,
                  float* C32, int64_t ldc32);
// G = Y^T Y (l x l) for Y d x l row-major with leading dimension l, through partial Gram matrices of
// row chunks (part: gram64_parts(d) x l x l scratch); the Cholesky factor G = R^T R of the sum of
// nparts matrices (upper triangles read) with R^{-1} (l x l, row-major); Rp: scratch of
// l (l + 1) / 2 + l doubles (the packed factor and its reciprocal diagonal)
int64_t gram64_parts(int64_t d);
int launch_gram64(hipStream_t st, const double* Y, int64_t d, int l, double* part, double* G);
int launch_chol_inv64(hipStream_t st, const double* part, int nparts, int l, double* Rp, double* Rinv, int* flag,
                      const int* gate = nullptr);  // gate (device, nullable): both kernels run only while *gate != 0
// The second CholeskyQR pass by symmetric orthogonalization when G = Q1^T Q1 = I + E has
// l max|E_ij| <= 1e-5 (Minv = I - E/2, plus 3 E^2/8 above 1e-7; *flag = 0, *use_chol = 0), else
// *use_chol = 1 for the gated Cholesky
int launch_lowdin64(hipStream_t st, const double* G, int l, double* Minv, int* flag, int* use_chol);
// one problem of a batched CholeskyQR2 (the buffers of cholqr2_64: Y d x l, Gp gram64_parts(d) l^2, G and
// Rinv l x l, Rp l (l + 1) / 2 + l, Q1 d x l, Q d x l with leading dimension ldq, QT l x d FP32 or null,
// flags[0..1] the two factorizations' breakdown flags)
struct CholJob {
  const double* Y;
  int64_t d;
  int l;
  double* Gp;
  double* G;
  double* Rp;
  double* Rinv;
  double* Q1;
  double* Q;
  int64_t ldq;
  float* QT;
  int* flags;
  int* gate;  // device int: the second pass takes the Cholesky (1) or the symmetric orthogonalization (0)
};
// CholeskyQR2 of nj problems at once (jobs: device array), eleven launches in all
int launch_cholqr2_batched(hipStream_t st, const CholJob* jobs, int nj, int64_t max_d, int max_l);
int launch_axpy64(hipStream_t st, int64_t count, double alpha, const double* x, double* y);
int launch_copy64(hipStream_t st, int64_t rows, int64_t cols, const double* src, int64_t lds, double* dst,
                  int64_t ldd);
int launch_transpose64to32(hipStream_t st, int64_t rows, int64_t cols, const double* src, int64_t lds, float* dst);
int launch_or_flags(hipStream_t st, const int* src, int count, int* dst);
// symmetric eigendecomposition B = V diag(theta) V^T (k_eig64.hip); work: eig64_work_len(l) doubles
int eig64_work_len(int l);
int launch_eig64(hipStream_t st, const double* B, int l, double* work, double* V, double* theta, int* order);
// one problem of a batched eigendecomposition (the arguments of launch_eig64)
struct Eig64Job {
  const double* B;
  int l;
  double* work;  // eig64_work_len(l) doubles
  double* V;
  double* theta;
  int* order;
};
// launch_eig64 for njobs problems at once, one workgroup per problem (jobs: device array)
int launch_eig64_batched(hipStream_t st, const Eig64Job* jobs, int njobs, int max_l);
// one problem of a batched lift (the arguments of launch_lift; U64 may be null)
struct LiftJob {
  const double* Q;
  int64_t d;
  int l;
  const double* V;
  const int* order;
  int k;
  const double* theta;
  double* U64;
  float* U32;
  float* UT32;
  double* lam;
  float* VkT;
};
int launch_lift_batched(hipStream_t st, const LiftJob* jobs, int njobs, int64_t max_elems);
// vector / small kernels
int launch_lift(hipStream_t st, const double* Q, int64_t d, int l, const double* V, const int* order, int k,
                const double* theta, double* U64, float* U32, float* UT32, double* lam, float* VkT);
// UD = U diag(D) and a copy of U, both gemm_wide_bt_rows(d) x ldu (ldu = gemm_wide_kpad(k)), zero past
// k and past d; scal = {1/s, sqrt(n lambda)/s}.
int launch_precond_setup(hipStream_t st, const double* lam, int k, double lambda, int64_t n, const float* U32,
                         int64_t d, float* UD, float* Up, int64_t ldu, double* scal, SolveState* state);
// zeroes up to three device buffers (sizes in bytes, multiples of 4; null buffers are skipped) in one launch
int launch_zero3(hipStream_t st, void* a, int64_t abytes, void* b, int64_t bbytes, void* c, int64_t cbytes);
int launch_premap(hipStream_t st, const float* UT, const float* U, const double* lam, int k, int64_t d,
                  double lambda, const float* wt, float* w, float* trace_row, double* tmp,
                  const SolveState* state);
// the two regularizations of the O~(ndk) budget from k sketched eigenvalues and state->beta_sum = ||X||_F^2
int launch_budget_lambda(hipStream_t st, const double* lam, int k, const SolveState* state, int64_t n, double* out);
// wt = P^{1/2} w (k <= 256; k = 0 copies), one workgroup
int launch_pmhalf_inv(hipStream_t st, const float* UT, const double* lam, int k, int64_t d, double lambda,
                      const float* w, float* wt);
int launch_rownorm(hipStream_t st, const float* X, int64_t n, int64_t d, int64_t ldx, float* out);
int launch_rownorm_bf16(hipStream_t st, const uint16_t* X, int64_t n, int64_t d, float* out);
int launch_copy_bf16(hipStream_t st, const float* X, int64_t n, int64_t d, int64_t ldx, uint16_t* out);
int launch_transpose_f32(hipStream_t st, const float* A, int64_t rows, int64_t cols, float* AT);
int launch_fill_scaled_identity(hipStream_t st, int64_t d, double alpha, int bf16, void* out, float* beta_reg);
int launch_grad_partial(hipStream_t st, const float* X, int64_t n, int64_t d, int64_t ldx, const float* y,
                        const float* w, float* part, double* rsq_part, int nwg, const SolveState* state);
int grad_num_workgroups(int64_t n, int64_t d);
int launch_grad_finish(hipStream_t st, const float* part, const double* rsq_part, int nwg, int64_t n, int64_t d,
                       const float* w, double lambda, const float* UT, const float* U, const double* lam, int k,
                       float* mu, double* g_tmp, double* tmp, SolveState* state, int stop_rule, double eps,
                       double f_star, float* wt_cur, const float* wt_prev, int first, int* host_stop);

// inner loop (one persistent launch per epoch)
struct InnerArgs {
  int64_t n, d;
  const void* Xt;      // data rows (index < n), leading dimension ldx
  int64_t ldx;
  const void* reg;     // regularizer rows (index >= n), leading dimension ldr
  int64_t ldr;
  const float* mu;     // snapshot gradient
  const int32_t* idx;  // m*b component indices
  const float* scale;  // m*b values 1/(n q_i)
  int64_t m;
  int b;
  double eta;
  int eta_from_state;  // 1: eta = step_scale * n / state->beta_sum
  double step_scale;
  int average;
  int W;               // cooperating workgroups
  int xcd_stride;      // blockIdx stride between cooperating workgroups
  int64_t slice;       // columns per workgroup (set by the launcher)
  uint32_t step_base;  // value of the step counters before this epoch
  float* wt;           // snapshot (in/out)
  float* wt_prev;      // copy of the incoming snapshot (nullable)
  uint64_t* xbuf;      // inner_xbuf_words(W) words: (step tag << 32) | partial dot product bits; zeroed per solve
  SolveState* state;
  int wave_rows;       // 0 = chosen from b and the slice width; 1, 2 or 4: waves split over rows;
                       // kInnerLookahead: the look-ahead kernel (k_inner_la.hip)
};
// Largest minibatch of the inner loop, and the exchange words its workgroups post (two step parities
// x up to 4 wave-rows x W workgroups x 64 rows = 2 W kInnerMaxB).
constexpr int kInnerMaxB = 256;
constexpr int kInnerLookahead = SCS_LOOKAHEAD;   // wave_rows value selecting the look-ahead kernel
inline int64_t inner_xbuf_words(int W) { return (int64_t)2 * W * kInnerMaxB; }
int launch_inner_epoch(hipStream_t st, InnerArgs& a, int bf16);
// wave-row count launch_inner_epoch uses for (b, d, W, requested wave_rows)
int inner_layout_wave_rows(int b, int64_t d, int W, int wave_rows);
int inner_default_workgroups(int64_t d);
// The look-ahead variant of the inner loop (the next step's dot products formed while the current
// exchange is in flight): same arguments and results up to rounding; needs b <= 64 and W >= d / 64.
bool inner_lookahead_fits(int b, int64_t d, int W);
int launch_inner_epoch_lookahead(hipStream_t st, InnerArgs& a, int bf16);

// ---------------------------------------------------------------- allocation-free entry (noalloc.hip)
// Looks up the device address of the fixed scratch array on `device` (which must be current); once per device.
int noalloc_scratch_init(int device);
size_t noalloc_full_gradient_bytes(int64_t n, int64_t d, int k);
int full_gradient_noalloc(int device, hipStream_t st, const float* X, int64_t n, int64_t d, int64_t ldx,
                          const float* y, const float* U, const double* lam, int k, double lambda, const float* wt,
                          float* grad_out, double* obj_out);

// ---------------------------------------------------------------- batched solves
// One problem of a batched solve; an array of these lives in device memory and every batched
// kernel finds its problem from its block index (flattened grids use the prefix arrays below).
struct BatchProb {
  const float* X;        // n x d, leading dimension ldx (the gradient pass streams X itself)
  int64_t n, d, ldx;
  const float* y;
  double lambda;
  const float* UT;       // k x d (FP32) and the Ritz values; k = 0: P = I
  const double* lam;
  int k;
  float* wt;             // snapshot w~ (in/out)
  float* wt_prev;
  float* w32;            // w = P^{-1/2} w~ at the snapshot
  float* mu;             // P^{-1/2}-mapped gradient (inner loop input)
  double* tmp;           // d doubles
  SolveState* state;
  float* gpart;          // nwg x d gradient partials
  double* grsq;          // nwg residual partials
  double* g64;           // grows x d first-level column sums (summed by the finalizer)
  int grows;             // 16 for the streaming pass, 1 when the sums come from the batched GEMMs
  int nwg;               // residual partials in grsq
  int stop_rule;
  double eps, f_star;
  const uint64_t* cum;   // cumulative integer sampling weights over N = n + d components
  int64_t N;
  const float* Z;        // n x k (X U~, leading dimension ldz) for the implicit inner loop, else unused
  int64_t ldz;
  int64_t draws;         // m b draws per epoch
  int32_t* idx;          // kSampleGroup epochs of draws
  float* scale;
  InnerArgs inner;       // idx / scale / step_base are set per epoch by the batched launchers
};
// flattened grids: prefix[p] = first unit of problem p, prefix[nprob] = total
int launch_premap_batched(hipStream_t st, const BatchProb* P, int nprob, int final_out, float* const* w_out);
int launch_grad_partial_batched(hipStream_t st, const BatchProb* P, int nprob, const int64_t* wg_prefix,
                                int64_t base, int64_t count, int64_t max_d, int vec4);
int launch_grad_finish_batched(hipStream_t st, const BatchProb* P, int nprob, const int64_t* cb_prefix,
                               int64_t total_cb, int first, int* done_count, int* host_stop, const int* clk = nullptr);
// implicit preconditioned rows (k_implicit.hip): one workgroup per problem; inner.Xt holds X itself
int launch_inner_implicit_batched(hipStream_t st, const BatchProb* P, int nprob, int64_t max_d, int max_k, int max_b,
                                  int epoch_slot, int64_t epoch, const int* clk = nullptr);
int launch_implicit_beta(hipStream_t st, const float* xnorm2, const float* Z, int64_t ldz, const float* UT,
                         const double* lam, int k, int64_t n, int64_t d, double lambda, float* beta);
int launch_grad_finalize_batched(hipStream_t st, const BatchProb* P, int nprob, int first, int* done_count,
                                 int* host_stop, const int* clk = nullptr);
// Shared-X gradient of many problems: R = X W^T (gemm), then R[i][p] -= Y[p % ny][i] with per-block
// residual sums rsq[p][blk]; then G (P x d, FP64) = sum over row chunks of the X^T R partials.
int launch_residual_batched(hipStream_t st, float* R, int64_t n, int P, const float* Y, int ny, int nblk,
                            double* rsq, Gate gate = Gate());
int launch_reduce_partials_t(hipStream_t st, const float* partial, int64_t nchunks, int64_t d, int Pc, double* G,
                             int64_t ldg, Gate gate = Gate());
int launch_sample_batched(hipStream_t st, const BatchProb* P, int nprob, const int64_t* draw_prefix,
                          int64_t total_draws, uint64_t seed, int epoch, int groups, const int* clk = nullptr);
int launch_inner_epoch_batched(hipStream_t st, const BatchProb* P, int nprob, int W, int64_t max_slice, int max_b,
                               int bf16, int epoch_slot, int64_t epoch, const int* clk = nullptr);
// Epochs of a batched or path solve replayed from a captured graph read their epoch number from a
// device clock: clk[0] = epoch, clk[1] = the epoch cap S. Kernels given a clock ignore their host
// epoch arguments (and skip epochs >= S, or > S for the gradient finish); index streams are drawn
// kEpochGroup epochs at a time, when the epoch number is a multiple of kEpochGroup.
constexpr int kEpochGroup = 8;
int launch_clock_set(hipStream_t st, int* clk, int epoch, int epochs);
int launch_clock_advance(hipStream_t st, int* clk);

// ---------------------------------------------------------------- the FP64 path (k_f64.hip)
constexpr int kF64MaxD = 4096;  // columns: one workgroup of 1024 threads, four columns each
constexpr int kF64MaxL = 136;   // sketch width k + p (the eigensolver's limit)
struct Inner64Args {
  int64_t n, d;
  const double* Xt;    // n data rows, stride ld
  const double* reg;   // d regularizer rows, stride ld
  int64_t ld;
  const int32_t* idx;  // m b component indices of the epoch
  const double* scale; // 1/(n q_i) per draw
  int64_t m;
  int b;
  const double* mu;    // full gradient at the snapshot (preconditioned coordinates)
  double* wt;          // the snapshot in, the next snapshot out
  double* wt_prev;     // receives the snapshot (nullable)
  double step_scale;   // eta = step_scale n / sum(beta), halved per rejected snapshot
  int average;
  SolveState* state;
};
int launch_f32_to_f64(hipStream_t st, int64_t count, const float* src, double* dst);
int launch_scale64(hipStream_t st, int64_t count, double alpha, double* x);
int launch_precond_setup64(hipStream_t st, const double* U, const double* lam, int k, int64_t d, double lambda,
                           double* UT, double* UDT, SolveState* state);
int launch_rows64(hipStream_t st, int64_t rows, const double* A, int64_t lda, const double* UDT, int k,
                  const double* base, int64_t ldb, int64_t d, const double* lam, double lambda, double alpha,
                  double* out, int64_t ldo, double* beta);
int grad64_workgroups(int64_t n);
int launch_grad64(hipStream_t st, const double* X, int64_t n, int64_t d, int64_t ldx, const double* y,
                  const double* w, int nwg, double* part, double* rsq, const SolveState* state);
int launch_finish64(hipStream_t st, const double* part, const double* rsq, int nwg, int64_t n, int64_t d,
                    const double* w, double lambda, const double* UT, const double* lam, int k, double* mu,
                    SolveState* state, int stop_rule, double eps, double f_star, double* wt, const double* wt_prev,
                    int first, int* host_stop);
int launch_premap64(hipStream_t st, const double* UT, const double* lam, int k, int64_t d, double lambda,
                    const double* wt, double* w, const SolveState* state);
int launch_inner64(hipStream_t st, const Inner64Args& a);

}  // namespace scs
