// The FP64 instantiation of the path (Alg. 1 and Alg. 3 with X, y, the preconditioned rows, the
// iterate and every sum in FP64), for problems whose columns fit one workgroup (d <= kF64MaxD).
// The sketch reuses the FP64 GEMM, CholeskyQR2 and eigensolver of the FP32 path, and the sampler its
// exact integer weights (quantized from FP64 beta here). The FP32 path spreads its wide problems
// over many cooperating workgroups; these kernels keep one problem's vectors in one workgroup:
//   rows64      x~_i = alpha (b_i / s + (D U~^T)^T a_i), one workgroup per row, with ||x~_i||^2
//               (the data rows: b = x_i, a = z_i = U~^T x_i, alpha = 1; the regularizer rows of
//               Alg. 3: b = e_j, a = U~^T e_j, alpha = sqrt(n lambda));
//   grad64      r = X w - y and the partial sums of X^T r per workgroup of rows (Alg. 1, the full
//               gradient at the snapshot);
//   finish64    g = X^T r / n + lambda w, mu = P^{-1/2} g, L(w), the certificate and the stop rules
//               (one workgroup);
//   premap64    w = P^{-1/2} w~ (one workgroup);
//   inner64     the m inner steps of one epoch, persistent in one workgroup (no cross-workgroup
//               exchange): the b dot products a_i^T (w - w_bar) one wave per row, then each thread
//               updates its columns of w - w_bar and of the running sum.
#include "scs_internal.h"

namespace scs {

namespace {

constexpr int kF64Block = 1024;  // threads of the one-workgroup kernels
constexpr int kF64Waves = kF64Block / 64;
constexpr int kF64Cols = kF64MaxD / kF64Block;  // columns per thread in the inner loop
constexpr int kRowBlock = 256;                   // threads of the row and gradient kernels
constexpr int kGradCols = kF64MaxD / kRowBlock;  // columns per thread in the gradient pass
constexpr int kGradRows = 64;                    // rows whose residuals one pass of grad64 stages
constexpr int kF64StageRows = 3072;              // doubles of LDS for the inner loop's staged rows

// Sum over a workgroup; every thread returns the same value (xor butterflies give every lane the
// same bits, and the wave sums are added in wave order).
__device__ __forceinline__ double block_sum64(double v, double* sred) {
  v = warp_sum_d(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sred[wave] = v;
  __syncthreads();
  double t = 0.0;
  for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += sred[q];
  return t;
}

__global__ void f32_to_f64_kernel(int64_t count, const float* src, double* dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) dst[e] = (double)src[e];
}

__global__ void scale64_kernel(int64_t count, double alpha, double* x) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) x[e] *= alpha;
}

// UT = U~^T and UDT = D U~^T (k x d) with D = diag(1/sqrt(lam_i + lambda) - 1/s), s = sqrt(lam_k + lambda)
// (Sec. 4.1, Eq. (condSketch): P^{-1/2} = I/s + U~ D U~^T).
__global__ void precond_setup64_kernel(const double* U, const double* lam, int k, int64_t d, double lambda,
                                       double* UT, double* UDT, SolveState* state) {
  const double s = sqrt(fmax(lam[k - 1], 0.0) + lambda);
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < (int64_t)k * d) {
    const int i = (int)(e / d);
    const int64_t j = e - (int64_t)i * d;
    const double u = U[j * k + i];
    UT[e] = u;
    UDT[e] = u * (1.0 / sqrt(fmax(lam[i], 0.0) + lambda) - 1.0 / s);
  }
  if (e == 0 && state) {
    state->s = s;
    state->lam_top = fmax(lam[0], 0.0);
  }
}

// out_i = alpha (base_i / s + UDT^T a_i) for row i = blockIdx.x (base = the identity when null; s = 1
// when k = 0), zero in the padding columns d .. ldo; beta[i] = ||out_i||^2.
__global__ __launch_bounds__(kRowBlock) void rows64_kernel(const double* A, int64_t lda, const double* UDT, int k,
                                                           const double* base, int64_t ldb, int64_t d,
                                                           const double* lam, double lambda, double alpha, double* out,
                                                           int64_t ldo, double* beta) {
  __shared__ double a_s[kF64MaxL];
  __shared__ double sred[kRowBlock / 64];
  const int64_t i = blockIdx.x;
  const double inv_s = k > 0 ? 1.0 / sqrt(fmax(lam[k - 1], 0.0) + lambda) : 1.0;
  for (int c = threadIdx.x; c < k; c += blockDim.x) a_s[c] = A[i * lda + c];
  __syncthreads();
  double sq = 0.0;
  for (int64_t j = threadIdx.x; j < ldo; j += blockDim.x) {
    double v = 0.0;
    if (j < d) {
      const double b = base ? base[i * ldb + j] : (j == i ? 1.0 : 0.0);
      double z = 0.0;
      for (int c = 0; c < k; ++c) z += a_s[c] * UDT[(int64_t)c * d + j];
      v = alpha * (b * inv_s + z);
      sq += v * v;
    }
    out[i * ldo + j] = v;
  }
  sq = block_sum64(sq, sred);
  if (threadIdx.x == 0 && beta) beta[i] = sq;
}

// Rows [r0, r1) of workgroup blockIdx.x: r_i = x_i^T w - y_i, part[wg][j] = sum_i r_i x_ij and
// rsq[wg] = sum_i r_i^2. Each pass stages kGradRows residuals (one wave per row, lanes over the
// columns), then every thread adds them into its kGradCols columns.
__global__ __launch_bounds__(kRowBlock) void grad64_kernel(const double* X, int64_t n, int64_t d, int64_t ldx,
                                                           const double* y, const double* w, int64_t rows_per_wg,
                                                           double* part, double* rsq, const SolveState* state) {
  if (state && state->done) return;
  __shared__ double w_s[kF64MaxD];
  __shared__ double r_s[kGradRows];
  __shared__ double sred[kRowBlock / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t j = threadIdx.x; j < d; j += blockDim.x) w_s[j] = w[j];
  double acc[kGradCols];
#pragma unroll
  for (int q = 0; q < kGradCols; ++q) acc[q] = 0.0;
  double rs = 0.0;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg;
  const int64_t r1 = r0 + rows_per_wg < n ? r0 + rows_per_wg : n;
  __syncthreads();
  for (int64_t rb = r0; rb < r1; rb += kGradRows) {
    const int nr = (int)(r1 - rb < kGradRows ? r1 - rb : kGradRows);
    // each wave takes rows wave, wave + 4, ...: four of them at a time, their loads in flight together
    for (int r4 = wave; r4 < nr; r4 += 4 * (kRowBlock / 64)) {
      double dot[4] = {0.0, 0.0, 0.0, 0.0};
      for (int64_t j = lane; j < d; j += 64) {
        const double wj = w_s[j];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int rr = r4 + u * (kRowBlock / 64);
          if (rr < nr) dot[u] += X[(rb + rr) * ldx + j] * wj;
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int rr = r4 + u * (kRowBlock / 64);
        const double t = warp_sum_d(dot[u]);
        if (lane == 0 && rr < nr) {
          const double r = t - y[rb + rr];
          r_s[rr] = r;
          rs += r * r;
        }
      }
    }
    __syncthreads();
#pragma unroll 4
    for (int rr = 0; rr < nr; ++rr) {
      const double r = r_s[rr];
      const double* x = X + (rb + rr) * ldx;
#pragma unroll
      for (int q = 0; q < kGradCols; ++q) {
        const int64_t j = threadIdx.x + (int64_t)q * kRowBlock;
        if (j < d) acc[q] += r * x[j];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < kGradCols; ++q) {
    const int64_t j = threadIdx.x + (int64_t)q * kRowBlock;
    if (j < d) part[(int64_t)blockIdx.x * d + j] = acc[q];
  }
  rs = block_sum64(rs, sred);
  if (threadIdx.x == 0) rsq[blockIdx.x] = rs;
}

// out_j = v_j / s + sum_i UT[i][j] D_i (sum_l UT[i][l] v_l) (P^{-1/2} v, Eq. (condSketch)) for v in
// LDS; k = 0 gives out = v. One workgroup; coef holds the k coefficients D_i U~_i^T v. Column j's
// output is emitted by the thread that last reads v_j, so emit may overwrite v in place.
template <typename EMIT>
__device__ __forceinline__ void pmhalf64(const double* UT, const double* lam, int k, int64_t d, double lambda,
                                         const double* v, double* coef, EMIT emit) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (k == 0) {
    for (int64_t j = threadIdx.x; j < d; j += blockDim.x) emit(j, v[j]);
    return;
  }
  const double s = sqrt(fmax(lam[k - 1], 0.0) + lambda);
  for (int i = wave; i < k; i += (int)(blockDim.x >> 6)) {
    double t = 0.0;
    for (int64_t j = lane; j < d; j += 64) t += UT[(int64_t)i * d + j] * v[j];
    t = warp_sum_d(t);
    if (lane == 0) coef[i] = t * (1.0 / sqrt(fmax(lam[i], 0.0) + lambda) - 1.0 / s);
  }
  __syncthreads();
  for (int64_t j = threadIdx.x; j < d; j += blockDim.x) {
    double z = 0.0;
    for (int i = 0; i < k; ++i) z += UT[(int64_t)i * d + j] * coef[i];
    emit(j, v[j] / s + z);
  }
}

// The finish of the full gradient at the snapshot w (= P^{-1/2} w~): g = (sum of the partials) / n
// + lambda w, mu = P^{-1/2} g, then the snapshot decision; mu is written on acceptance, the previous
// w~ restored on rejection. host_stop as in the FP32 finish.
__global__ __launch_bounds__(kF64Block) void finish64_kernel(const double* part, const double* rsq, int nwg,
                                                             int64_t n, int64_t d, const double* w, double lambda,
                                                             const double* UT, const double* lam, int k, double* mu,
                                                             SolveState* state, int stop_rule, double eps,
                                                             double f_star, double* wt, const double* wt_prev,
                                                             int first, int* host_stop) {
  if (state->done) {
    if (host_stop && threadIdx.x == 0) __hip_atomic_store(host_stop, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    return;
  }
  __shared__ double g_s[kF64MaxD];  // g, then mu in place (each column's output replaces its own input)
  __shared__ double coef[kF64MaxL];
  __shared__ double sred[kF64Waves];
  __shared__ int s_action;
  for (int64_t j = threadIdx.x; j < d; j += blockDim.x) {
    double a = 0.0;
    for (int q = 0; q < nwg; ++q) a += part[(int64_t)q * d + j];
    g_s[j] = a / (double)n + lambda * w[j];
  }
  __syncthreads();
  pmhalf64(UT, lam, k, d, lambda, g_s, coef, [&](int64_t j, double x) { g_s[j] = x; });
  double gn = 0.0, wn = 0.0, rs = 0.0;
  for (int64_t j = threadIdx.x; j < d; j += blockDim.x) {
    gn += g_s[j] * g_s[j];
    wn += w[j] * w[j];
  }
  for (int q = threadIdx.x; q < nwg; q += blockDim.x) rs += rsq[q];
  gn = block_sum64(gn, sred);
  wn = block_sum64(wn, sred);
  rs = block_sum64(rs, sred);
  if (threadIdx.x == 0)
    s_action = snapshot_decision(state, rs / (2.0 * (double)n) + 0.5 * lambda * wn, gn, lam, k, lambda, first,
                                 stop_rule, eps, f_star);
  __syncthreads();
  const int action = s_action;
  if (action == 2 || action == 4)
    for (int64_t j = threadIdx.x; j < d; j += blockDim.x) wt[j] = wt_prev[j];
  if (action == 0 || action == 1)
    for (int64_t j = threadIdx.x; j < d; j += blockDim.x) mu[j] = g_s[j];
  if (host_stop && threadIdx.x == 0)
    __hip_atomic_store(host_stop, (action == 1 || action == 2 || action == 3) ? 1 : 2, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_SYSTEM);
}

// w = P^{-1/2} w~ (the map back of Alg. 3's output, and the gradient's evaluation point).
__global__ __launch_bounds__(kF64Block) void premap64_kernel(const double* UT, const double* lam, int k, int64_t d,
                                                             double lambda, const double* wt, double* w,
                                                             const SolveState* state) {
  if (state && state->done) return;
  __shared__ double v_s[kF64MaxD];
  __shared__ double coef[kF64MaxL];
  for (int64_t j = threadIdx.x; j < d; j += blockDim.x) v_s[j] = wt[j];
  __syncthreads();
  pmhalf64(UT, lam, k, d, lambda, v_s, coef, [&](int64_t j, double x) { w[j] = x; });
}

// One epoch of Alg. 1's inner loop on the n + d rows a_i (data rows Xt, then the regularizer rows
// reg, one stride ld): with delta = w - w_bar, step t draws i_1 .. i_b and sets
//   delta <- delta - eta ((1/b) sum_j scale_j (a_{i_j}^T delta) a_{i_j} + mu),
// scale_j = 1/(n q_{i_j}) (the variance-reduced direction divided by N q_i, times N/n for the
// N/n of each component), and adds delta to the running sum; at the end w~ <- w_bar + (sum / m)
// (average) or w_bar + delta (last iterate). eta = c n / sum(beta), halved per rejected snapshot.
// Step t: wave w forms the dot products of rows j = w, w + 16, ... (lanes over the columns) and, when
// b d fits, stages the rows in LDS; after a barrier each thread updates its columns (c = thread +
// NT q). PR > 0 (b <= (NT / 64) PR, d <= 64 PQ, the rows staged): each wave holds its rows of step t + 1 in
// registers, loaded during step t together with the indices of step t + 2, through global-address
// pointers so that the barriers do not wait for them.
typedef __attribute__((address_space(1))) const double gdouble;
typedef __attribute__((address_space(1))) const int32_t gint32;

// NT threads (NT / 64 waves), CPT columns per thread: d <= NT CPT.
template <int PR, int PQ, int NT, int CPT>
__global__ __launch_bounds__(NT) void inner64_kernel(Inner64Args a) {
  constexpr int kWaves = NT / 64;
  if (a.state->done) return;
  __shared__ double dl_s[kF64MaxD];
  __shared__ double rows_s[kF64StageRows];  // the step's b rows when b d fits, for the update phase
  __shared__ double coef[kInnerMaxB];
  __shared__ int row_s[kInnerMaxB];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t d = a.d, N = a.n + a.d;
  const int b = a.b;
  const bool staged = PR > 0 || (int64_t)b * d <= kF64StageRows;
  const double eta = ldexp(a.step_scale * (double)a.n / a.state->beta_sum, -a.state->backoffs);
  const double inv_b = 1.0 / (double)b;
  double w0[CPT], muv[CPT], dl[CPT], sm[CPT];
#pragma unroll
  for (int q = 0; q < CPT; ++q) {
    const int64_t c = threadIdx.x + (int64_t)q * NT;
    w0[q] = c < d ? a.wt[c] : 0.0;
    muv[q] = c < d ? a.mu[c] : 0.0;
    dl[q] = 0.0;
    sm[q] = 0.0;
    if (c < d) dl_s[c] = 0.0;
  }
  // a caller's index stream is clamped as the scales are
  auto clampi = [&](int64_t i) { return i < 0 ? (int64_t)0 : i >= N ? N - 1 : i; };
  auto rowp = [&](int64_t i) { return i < a.n ? a.Xt + i * a.ld : a.reg + (i - a.n) * a.ld; };
  // the update phase of step t, once coef and (when staged) rows_s hold the step
  auto update = [&]() {
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const int64_t c = threadIdx.x + (int64_t)q * NT;
      if (c < d) {
        double v = 0.0;
        if (staged) {
          for (int j = 0; j < b; ++j) v += coef[j] * rows_s[j * d + c];
        } else {
          for (int j = 0; j < b; ++j) v += coef[j] * rowp(row_s[j])[c];
        }
        dl[q] -= eta * (v * inv_b + muv[q]);
        sm[q] += dl[q];
        dl_s[c] = dl[q];
      }
    }
  };
  __syncthreads();
  if constexpr (PR == 0) {
    for (int64_t t = 0; t < a.m; ++t) {
      const int32_t* idx = a.idx + t * b;
      const double* sc = a.scale + t * b;
      for (int j = wave; j < b; j += kWaves) {
        const int64_t i = clampi(idx[j]);
        const double* row = rowp(i);
        double dot = 0.0;
        for (int64_t c = lane; c < d; c += 64) {
          const double x = row[c];
          dot += x * dl_s[c];
          if (staged) rows_s[j * d + c] = x;
        }
        dot = warp_sum_d(dot);
        if (lane == 0) {
          coef[j] = sc[j] * dot;
          row_s[j] = (int)i;
        }
      }
      __syncthreads();
      update();
      __syncthreads();
    }
  } else {
    const gint32* gidx = (const gint32*)a.idx;
    const gdouble* gsc = (const gdouble*)a.scale;
    auto load = [&](int64_t t, const int64_t (&ii)[PR], double (&x)[PR][PQ], double (&scv)[PR]) {
#pragma unroll
      for (int r = 0; r < PR; ++r) {
        const int j = wave + kWaves * r;
        const gdouble* row = (const gdouble*)rowp(ii[r]);
        scv[r] = j < b ? gsc[t * b + j] : 0.0;
#pragma unroll
        for (int q = 0; q < PQ; ++q) {
          const int64_t c = lane + 64 * q;
          x[r][q] = (j < b && c < d) ? row[c] : 0.0;
        }
      }
    };
    auto indices = [&](int64_t t, int64_t (&ii)[PR]) {
#pragma unroll
      for (int r = 0; r < PR; ++r) {
        const int j = wave + kWaves * r;
        ii[r] = (t < a.m && j < b) ? clampi(gidx[t * b + j]) : 0;
      }
    };
    int64_t i_cur[PR], i_next[PR];
    double x_cur[PR][PQ], s_cur[PR];
    indices(0, i_cur);
    indices(1, i_next);
    if (a.m > 0) load(0, i_cur, x_cur, s_cur);
    for (int64_t t = 0; t < a.m; ++t) {
      double x_next[PR][PQ], s_next[PR];
      int64_t i_after[PR];
      if (t + 1 < a.m) load(t + 1, i_next, x_next, s_next);
      indices(t + 2, i_after);
#pragma unroll
      for (int r = 0; r < PR; ++r) {
        const int j = wave + kWaves * r;
        if (j < b) {  // uniform over the wave
          double dot = 0.0;
#pragma unroll
          for (int q = 0; q < PQ; ++q) {
            const int64_t c = lane + 64 * q;
            if (c < d) {
              dot += x_cur[r][q] * dl_s[c];
              rows_s[j * d + c] = x_cur[r][q];
            }
          }
          dot = warp_sum_d(dot);
          if (lane == 0) coef[j] = s_cur[r] * dot;
        }
      }
      __syncthreads();
      update();
      __syncthreads();
#pragma unroll
      for (int r = 0; r < PR; ++r) {
        s_cur[r] = s_next[r];
        i_next[r] = i_after[r];
#pragma unroll
        for (int q = 0; q < PQ; ++q) x_cur[r][q] = x_next[r][q];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < CPT; ++q) {
    const int64_t c = threadIdx.x + (int64_t)q * NT;
    if (c < d) {
      if (a.wt_prev) a.wt_prev[c] = w0[q];
      a.wt[c] = w0[q] + (a.average ? sm[q] / (double)a.m : dl[q]);
    }
  }
  if (threadIdx.x == 0) {
    a.state->epochs += 1;
    a.state->eta = eta;
  }
}

}  // namespace

int launch_f32_to_f64(hipStream_t st, int64_t count, const float* src, double* dst) {
  if (count <= 0) return SCS_OK;
  f32_to_f64_kernel<<<dim3((unsigned)cdiv(count, 256)), dim3(256), 0, st>>>(count, src, dst);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_scale64(hipStream_t st, int64_t count, double alpha, double* x) {
  if (count <= 0) return SCS_OK;
  scale64_kernel<<<dim3((unsigned)cdiv(count, 256)), dim3(256), 0, st>>>(count, alpha, x);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_precond_setup64(hipStream_t st, const double* U, const double* lam, int k, int64_t d, double lambda,
                           double* UT, double* UDT, SolveState* state) {
  if (k < 1) return SCS_EINVAL;
  precond_setup64_kernel<<<dim3((unsigned)cdiv((int64_t)k * d, 256)), dim3(256), 0, st>>>(U, lam, k, d, lambda, UT,
                                                                                           UDT, state);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_rows64(hipStream_t st, int64_t rows, const double* A, int64_t lda, const double* UDT, int k,
                  const double* base, int64_t ldb, int64_t d, const double* lam, double lambda, double alpha,
                  double* out, int64_t ldo, double* beta) {
  if (rows <= 0) return SCS_OK;
  if (k < 0 || k > kF64MaxL || d > kF64MaxD || ldo < d || (k > 0 && (!A || !UDT || !lam)) || (!base && rows > d))
    return SCS_EINVAL;
  rows64_kernel<<<dim3((unsigned)rows), dim3(kRowBlock), 0, st>>>(A, lda, UDT, k, base, ldb, d, lam, lambda, alpha,
                                                                  out, ldo, beta);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int grad64_workgroups(int64_t n) {
  // one workgroup per kGradRows rows up to 256 workgroups (the finish adds the partials of every
  // workgroup for each column), more rows per workgroup beyond
  const int64_t w = cdiv(n, (int64_t)kGradRows);
  return (int)(w < 1 ? 1 : w > 256 ? 256 : w);
}

int launch_grad64(hipStream_t st, const double* X, int64_t n, int64_t d, int64_t ldx, const double* y,
                  const double* w, int nwg, double* part, double* rsq, const SolveState* state) {
  if (d > kF64MaxD || nwg < 1) return SCS_EINVAL;
  const int64_t per = cdiv(n, (int64_t)nwg);
  grad64_kernel<<<dim3((unsigned)nwg), dim3(kRowBlock), 0, st>>>(X, n, d, ldx, y, w, per, part, rsq, state);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_finish64(hipStream_t st, const double* part, const double* rsq, int nwg, int64_t n, int64_t d,
                    const double* w, double lambda, const double* UT, const double* lam, int k, double* mu,
                    SolveState* state, int stop_rule, double eps, double f_star, double* wt, const double* wt_prev,
                    int first, int* host_stop) {
  if (d > kF64MaxD || k > kF64MaxL) return SCS_EINVAL;
  finish64_kernel<<<1, kF64Block, 0, st>>>(part, rsq, nwg, n, d, w, lambda, UT, lam, k, mu, state, stop_rule, eps,
                                           f_star, wt, wt_prev, first, host_stop);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_premap64(hipStream_t st, const double* UT, const double* lam, int k, int64_t d, double lambda,
                    const double* wt, double* w, const SolveState* state) {
  if (d > kF64MaxD || k > kF64MaxL) return SCS_EINVAL;
  premap64_kernel<<<1, kF64Block, 0, st>>>(UT, lam, k, d, lambda, wt, w, state);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_inner64(hipStream_t st, const Inner64Args& a) {
  if (a.d > kF64MaxD || a.b < 1 || a.b > kInnerMaxB || a.m < 0) return SCS_EINVAL;
  const bool fits = (int64_t)a.b * a.d <= kF64StageRows;
  // (four waves with two rows each were slower at b = 8, d = 100: 1.49 against 1.37 us per step)
  if (fits && a.b <= kF64Waves && a.d <= 128) inner64_kernel<1, 2, kF64Block, kF64Cols><<<1, kF64Block, 0, st>>>(a);
  else if (fits && a.b <= 2 * kF64Waves && a.d <= 256)
    inner64_kernel<2, 4, kF64Block, kF64Cols><<<1, kF64Block, 0, st>>>(a);
  else inner64_kernel<0, 0, kF64Block, kF64Cols><<<1, kF64Block, 0, st>>>(a);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

}  // namespace scs
