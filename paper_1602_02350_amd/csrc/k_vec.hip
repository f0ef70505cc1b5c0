// Small kernels on d-vectors and k-vectors around the two streaming passes:
//  * the preconditioner on a vector, P^{-1/2} v = v/s + U~ (D (U~^T v)) (Eq. (condSketch)),
//    used both to evaluate the gradient at w = P^{-1/2} w~ and to return w (Eq. (condRidge));
//    because the same routine produces the point where the gradient is evaluated and the
//    returned weights, rounding in U~ moves neither the fixed point nor the output;
//  * the finish of the full-gradient pass (FP64 cross-workgroup sums, mu = P^{-1/2} g, the
//    objective, the stop rules and divergence handling);
//  * row norms, BF16 copies, the scaled identity (regularizer rows of plain SVRG),
//    lifting Ritz vectors (U~ = Q V_k) and the preconditioner's scalars.
#include "scs_internal.h"

namespace scs {

namespace {

constexpr int kVecThreads = 1024;
constexpr int kMaxPmhalfInvK = 256;
constexpr int kVecWaves = kVecThreads / 64;

__device__ __forceinline__ double block_sum_d(double v, double* sred) {
  v = wave_sum_d_fast(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sred[wave] = v;
  __syncthreads();
  double t = 0.0;
  for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += sred[q];
  return t;
}

// out_j = v_j/s + sum_i UT[i][j] D_i (sum_l UT[i][l] v_l); k = 0 gives out = v.
// UT is k x d (FP32), the sums are FP64; one workgroup, so the result is deterministic. v is staged
// in LDS (vs, kVsMax doubles) when it fits; tbuf holds the k coefficients. Phase 1 gives each wave
// R rows of UT at a time and phase 2 four threads to each four consecutive columns (a quarter of the
// rows each), with float4 loads when the rows of UT are 16-byte aligned, so every lane keeps many
// independent loads in flight.
// emit(j, value) receives out_j.
constexpr int kVsMax = 4096;
constexpr int kApplyR = 4;  // rows of UT per wave in phase 1

// Phase 1 with float4 loads for rows i0 .. i0 + 3 (one wave; d a multiple of 4, UT 16-byte aligned):
// tb[i] = (sum_j UT[i][j] v_j) (1/sqrt(lam_i + lambda) - 1/s). Each lane takes the column quads
// lane, lane + 64, ... in order, four per pass with all 16 float4 loads issued before the first is
// used (clamped indices keep them unconditional); the lanes' sums are then added across the wave.
template <typename VJ>
__device__ __forceinline__ void pmhalf_rows_v4(const float* __restrict__ UT, const double* __restrict__ lam, int k,
                                               int64_t d, double lambda, double s, int i0, int lane, VJ vj,
                                               double* tb) {
  constexpr int R = kApplyR, S = 4;
  const int d4 = (int)(d >> 2);
  double acc[R] = {0.0, 0.0, 0.0, 0.0};
  for (int jb = 0; jb < d4; jb += 64 * S) {
    float4 u[R][S];
#pragma unroll
    for (int q = 0; q < S; ++q) {
      const int j4 = jb + lane + 64 * q;
      const int jc = j4 < d4 ? j4 : d4 - 1;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int ir = i0 + r < k ? i0 + r : k - 1;
        u[r][q] = reinterpret_cast<const float4*>(UT + (int64_t)ir * d)[jc];
      }
    }
#pragma unroll
    for (int q = 0; q < S; ++q) {
      const int j4 = jb + lane + 64 * q;
      if (j4 < d4) {
        const double v0 = vj(4 * j4), v1 = vj(4 * j4 + 1), v2 = vj(4 * j4 + 2), v3 = vj(4 * j4 + 3);
#pragma unroll
        for (int r = 0; r < R; ++r)
          if (i0 + r < k)
            acc[r] += (double)u[r][q].x * v0 + (double)u[r][q].y * v1 + (double)u[r][q].z * v2 +
                      (double)u[r][q].w * v3;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    double t = wave_sum_d_fast(acc[r]);
    if (lane == 0 && i0 + r < k) tb[i0 + r] = t * (1.0 / sqrt(fmax(lam[i0 + r], 0.0) + lambda) - 1.0 / s);
  }
}

// Phase 2 with float4 loads for column quad j4: four consecutive lanes (part = lane & 3) each sum
// every fourth row of UT, in groups of 16 rows whose loads are issued together, and the four parts
// are combined as (p0 + p1) + (p2 + p3); the lane with part 0 emits out_j = v_j/s + the sum for the
// quad's four columns. Every lane of the wave must call it (j4 >= d4 contributes nothing).
template <typename VJ, typename EMIT>
__device__ __forceinline__ void pmhalf_quad_v4(const float* __restrict__ UT, const double* tb, int k, int64_t d,
                                               double s, int j4, int part, VJ vj, EMIT emit) {
  const int d4 = (int)(d >> 2);
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  if (j4 < d4) {
    constexpr int NB = 16;
    for (int ib = part; ib < k; ib += 4 * NB) {
      float4 u[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const int i = ib + 4 * q < k ? ib + 4 * q : k - 1;
        u[q] = reinterpret_cast<const float4*>(UT + (int64_t)i * d)[j4];
      }
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        if (ib + 4 * q < k) {
          const double t = tb[ib + 4 * q];
          a0 += (double)u[q].x * t;
          a1 += (double)u[q].y * t;
          a2 += (double)u[q].z * t;
          a3 += (double)u[q].w * t;
        }
      }
    }
  }
  a0 += __shfl_xor(a0, 1);
  a1 += __shfl_xor(a1, 1);
  a2 += __shfl_xor(a2, 1);
  a3 += __shfl_xor(a3, 1);
  a0 += __shfl_xor(a0, 2);
  a1 += __shfl_xor(a1, 2);
  a2 += __shfl_xor(a2, 2);
  a3 += __shfl_xor(a3, 2);
  if (j4 < d4 && part == 0) {
    emit(4 * j4, vj(4 * j4) / s + a0);
    emit(4 * j4 + 1, vj(4 * j4 + 1) / s + a1);
    emit(4 * j4 + 2, vj(4 * j4 + 2) / s + a2);
    emit(4 * j4 + 3, vj(4 * j4 + 3) / s + a3);
  }
}

template <typename VIN, typename EMIT>
__device__ __forceinline__ void pmhalf_apply_block(const float* __restrict__ UT, const double* __restrict__ lam, int k, int64_t d,
                                   double lambda, const VIN* __restrict__ v, double* vs, double* tbuf, EMIT emit) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);  // uniform: scalar loops
  const int dd = (int)d;
  const bool staged = dd <= kVsMax;
  if (staged) {
    for (int j = threadIdx.x; j < dd; j += blockDim.x) vs[j] = (double)v[j];
    __syncthreads();
  }
  auto vj = [&](int j) { return staged ? vs[j] : (double)v[j]; };
  if (k == 0) {
    for (int j = threadIdx.x; j < dd; j += blockDim.x) emit(j, vj(j));
    __syncthreads();
    return;
  }
  const double s = sqrt(fmax(lam[k - 1], 0.0) + lambda);
  const bool v4 = (dd & 3) == 0 && (reinterpret_cast<uintptr_t>(UT) & 15) == 0;
  const int d4 = dd >> 2;
  constexpr int R = kApplyR;  // rows of UT per wave and pass
  const int nwave = (int)blockDim.x >> 6;
  for (int i0 = wave * R; i0 < k; i0 += nwave * R) {
    if (v4) {
      pmhalf_rows_v4(UT, lam, k, d, lambda, s, i0, lane, vj, tbuf);
      continue;
    }
    double acc[R] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int j = lane; j < dd; j += 64) {
      const double x = vj(j);
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (i0 + r < k) acc[r] += (double)UT[(int64_t)(i0 + r) * d + j] * x;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      double t = wave_sum_d_fast(acc[r]);
      if (lane == 0 && i0 + r < k) tbuf[i0 + r] = t * (1.0 / sqrt(fmax(lam[i0 + r], 0.0) + lambda) - 1.0 / s);
    }
  }
  __syncthreads();
  if (v4) {
    // four threads per column quad
    const int part = threadIdx.x & 3;
    for (int j4base = 0; j4base < d4; j4base += (int)blockDim.x >> 2)
      pmhalf_quad_v4(UT, tbuf, k, d, s, j4base + ((int)threadIdx.x >> 2), part, vj, emit);
  } else {
    for (int j = threadIdx.x; j < dd; j += blockDim.x) {
      double acc = 0.0;
#pragma unroll 16
      for (int i = 0; i < k; ++i) acc += (double)UT[(int64_t)i * d + j] * tbuf[i];
      emit(j, vj(j) / s + acc);
    }
  }
  __syncthreads();
}

__device__ __forceinline__ void premap_body(const float* UT, const double* lam, int k, int64_t d, double lambda,
                                            const float* wt, float* w, float* trace_row) {
  __shared__ double tbuf[256];
  __shared__ double vs[kVsMax];
  pmhalf_apply_block<float>(UT, lam, k, d, lambda, wt, vs, tbuf, [&](int j, double x) {
    const float f = (float)x;
    w[j] = f;
    if (trace_row) trace_row[j] = f;
  });
}

__global__ __launch_bounds__(kVecThreads) void premap_kernel(const float* UT, const double* lam, int k, int64_t d,
                                                             double lambda, const float* wt, float* w,
                                                             float* trace_row, double* tmp,
                                                             const SolveState* state) {
  (void)tmp;
  if (state && state->done) return;
  premap_body(UT, lam, k, d, lambda, wt, w, trace_row);
}

// w~ = P^{1/2} w = s w + U~ diag(sqrt(lam_i + lambda) - s) U~^T w, the inverse of the output map
// w = P^{-1/2} w~ (Eq. (condSketch) with the powers 1/2): a start point given in the original space
// becomes the solver's own variable. One workgroup, FP64 arithmetic on FP32 inputs; k = 0 copies w.
__global__ __launch_bounds__(256) void pmhalf_inv_kernel(const float* UT, const double* lam, int k, int64_t d,
                                                         double lambda, const float* w, float* wt) {
  __shared__ double coef[kMaxPmhalfInvK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double s = k > 0 ? sqrt(fmax(lam[k - 1], 0.0) + lambda) : 1.0;
  for (int i = wave; i < k; i += 4) {
    double acc = 0.0;
    for (int64_t j = lane; j < d; j += 64) acc += (double)UT[(int64_t)i * d + j] * (double)w[j];
    acc = wave_sum_d_fast(acc);
    if (lane == 0) coef[i] = (sqrt(fmax(lam[i], 0.0) + lambda) - s) * acc;
  }
  __syncthreads();
  for (int64_t j = tid; j < d; j += 256) {
    double v = s * (double)w[j];
    for (int i = 0; i < k; ++i) v += (double)UT[(int64_t)i * d + j] * coef[i];
    wt[j] = (float)v;
  }
}

// One workgroup per problem: w = P^{-1/2} w~ at the snapshot (skipped once a problem is done), or,
// with final_out, the returned weights of every problem.
__global__ __launch_bounds__(kVecThreads) void premap_batched_kernel(const BatchProb* P, int final_out,
                                                                     float* const* w_out) {
  const BatchProb& q = P[blockIdx.x];
  if (final_out) {
    premap_body(q.UT, q.lam, q.k, q.d, q.lambda, q.wt, w_out[blockIdx.x], nullptr);
  } else {
    if (q.state->done) return;
    premap_body(q.UT, q.lam, q.k, q.d, q.lambda, q.wt, q.w32, nullptr);
  }
}

// First level of the cross-workgroup sum of the gradient partials, in FP64 and a fixed order:
// workgroup (bx, by) sums partial rows [by R, (by+1) R) of columns [64 bx, 64 bx + 64) into
// g2[by][j]; grad_finalize adds the kColSplit rows of g2 in order.
constexpr int kColSplit = 16;

__device__ __forceinline__ void colreduce_body(const float* part, int nwg, int64_t d, double* g2, int64_t bx, int by) {
  __shared__ double sacc[4][64];
  const int c = threadIdx.x & 63, rs = threadIdx.x >> 6;
  const int64_t j = bx * 64 + c;
  const int R = (nwg + kColSplit - 1) / kColSplit;
  const int r0 = by * R, r1 = r0 + R < nwg ? r0 + R : nwg;
  double acc = 0.0;
  if (j < d) {
#pragma unroll 4
    for (int q = r0 + rs; q < r1; q += 4) acc += (double)part[(int64_t)q * d + j];
  }
  sacc[rs][c] = acc;
  __syncthreads();
  if (rs == 0 && j < d) g2[(int64_t)by * d + j] = ((sacc[0][c] + sacc[1][c]) + sacc[2][c]) + sacc[3][c];
}

__global__ __launch_bounds__(256) void grad_colreduce_kernel(const float* part, int nwg, int64_t d, double* g2,
                                                             const SolveState* state) {
  if (state && state->done) return;
  colreduce_body(part, nwg, d, g2, blockIdx.x, blockIdx.y);
}

// problem p owns column blocks [cb_prefix[p], cb_prefix[p+1]) of grid dimension x
__global__ __launch_bounds__(256) void grad_colreduce_batched_kernel(const BatchProb* P, int nprob,
                                                                     const int64_t* cb_prefix) {
  const int p = find_prob(cb_prefix, nprob, blockIdx.x);
  const BatchProb& q = P[p];
  if (q.state->done) return;
  colreduce_body(q.gpart, q.nwg, q.d, q.g64, blockIdx.x - cb_prefix[p], blockIdx.y);
}

// g_j = (1/n) sum of the grows partial rows of column j (fixed order) + lambda w_j
__device__ __forceinline__ double grad_entry(const double* g_in, int grows, int64_t j, int64_t d, int64_t n,
                                             double lambda, const float* w) {
  double acc = 0.0;
  if (grows == kColSplit) {
#pragma unroll
    for (int q = 0; q < kColSplit; ++q) acc += g_in[(int64_t)q * d + j];
  } else {
    for (int q = 0; q < grows; ++q) acc += g_in[(int64_t)q * d + j];
  }
  return acc / (double)n + lambda * (double)w[j];
}

__device__ __forceinline__ int finalize_tail(const double* rsq_part, int nwg, int64_t n, int64_t d, const float* w,
                                             double lambda, const double* lam, int k, float* mu, const double* tmp,
                                             SolveState* state, int stop_rule, double eps, double f_star,
                                             float* wt_cur, const float* wt_prev, int first);

// Finish of the gradient at the snapshot for one problem (one workgroup); returns the action taken
// (0 continue, 1 converged, 2 diverged and restored, 3 non-finite input), the same in every thread.
__device__ __forceinline__ int finalize_body(const double* g_in, int grows, const double* rsq_part, int nwg, int64_t n, int64_t d,
                             const float* w, double lambda, const float* UT, const double* lam, int k, float* mu,
                             double* tmp, SolveState* state, int stop_rule, double eps, double f_star, float* wt_cur,
                             const float* wt_prev, int first) {
  __shared__ double tbuf[256];
  __shared__ double vs[kVsMax];
  // g = (1/n) sum of the partial rows (fixed order) + lambda w, written over the first row of g2
  double* g = const_cast<double*>(g_in);
  for (int64_t j = threadIdx.x; j < d; j += blockDim.x) g[j] = grad_entry(g_in, grows, j, d, n, lambda, w);
  __syncthreads();
  // mu = P^{-1/2} g
  pmhalf_apply_block<double>(UT, lam, k, d, lambda, g, vs, tbuf, [&](int j, double x) { tmp[j] = x; });
  return finalize_tail(rsq_part, nwg, n, d, w, lambda, lam, k, mu, tmp, state, stop_rule, eps, f_star, wt_cur,
                       wt_prev, first);
}

// The rest of the finish once tmp holds mu = P^{-1/2} g: norms, objective, stop rules, the action
// taken (same in every thread), and mu in FP32 or the restored snapshot.
__device__ __forceinline__ int finalize_tail(const double* rsq_part, int nwg, int64_t n, int64_t d, const float* w,
                                             double lambda, const double* lam, int k, float* mu, const double* tmp,
                                             SolveState* state, int stop_rule, double eps, double f_star,
                                             float* wt_cur, const float* wt_prev, int first) {
  __shared__ double sred[kVecWaves];
  __shared__ int s_action;
  double gn = 0.0, wn = 0.0;
  for (int64_t j = threadIdx.x; j < d; j += blockDim.x) {
    double m = tmp[j];
    gn += m * m;
    double wj = (double)w[j];
    wn += wj * wj;
  }
  gn = block_sum_d(gn, sred);
  wn = block_sum_d(wn, sred);
  double rs = 0.0;
  for (int q = threadIdx.x; q < nwg; q += blockDim.x) rs += rsq_part[q];
  rs = block_sum_d(rs, sred);
  if (threadIdx.x == 0)
    s_action = snapshot_decision(state, rs / (2.0 * (double)n) + 0.5 * lambda * wn, gn, lam, k, lambda, first,
                                 stop_rule, eps, f_star);
  __syncthreads();
  if ((s_action == 2 || s_action == 4) && wt_prev) {
    for (int64_t j = threadIdx.x; j < d; j += blockDim.x) wt_cur[j] = wt_prev[j];
  }
  if (s_action == 0 || s_action == 1) {
    for (int64_t j = threadIdx.x; j < d; j += blockDim.x) mu[j] = (float)tmp[j];
  }
  return s_action;
}

__global__ __launch_bounds__(kVecThreads) void grad_finalize_kernel(
    const double* g_in, const double* rsq_part, int nwg, int64_t n, int64_t d, const float* w, double lambda,
    const float* UT, const double* lam, int k, float* mu, double* tmp, SolveState* state, int stop_rule, double eps,
    double f_star, float* wt_cur, const float* wt_prev, int first, int* host_stop) {
  // host_stop (host-pinned, may be null) receives 1 once no further epoch will change anything, so the
  // host can stop enqueuing epochs, else 2 (so that 0 still means "not written yet"); it is a plain
  // system-scope store from one lane
  if (state->done) {
    if (host_stop && threadIdx.x == 0) __hip_atomic_store(host_stop, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    return;
  }
  const int action = finalize_body(g_in, kColSplit, rsq_part, nwg, n, d, w, lambda, UT, lam, k, mu, tmp, state,
                                   stop_rule, eps, f_star, wt_cur, wt_prev, first);
  if (host_stop && threadIdx.x == 0)
    __hip_atomic_store(host_stop, (action == 1 || action == 2 || action == 3) ? 1 : 2, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_SYSTEM);
}

// One workgroup per problem. A problem that finishes in this launch adds one to done_count; the
// workgroup that brings it to nprob sets the host-pinned flag (the host then stops enqueuing).
__global__ __launch_bounds__(kVecThreads) void grad_finalize_batched_kernel(const BatchProb* P, int nprob, int first,
                                                                            int* done_count, int* host_stop,
                                                                            const int* clk) {
  if (clk) {  // epochs replayed from a graph: the epoch number is on the device; host_stop is the flag array
    const int s = clk[0];
    if (s > clk[1]) return;
    first = s == 0;
    host_stop = host_stop ? host_stop + s : nullptr;
  }
  const BatchProb& q = P[blockIdx.x];
  if (q.state->done) return;
  const int action = finalize_body(q.g64, q.grows, q.grsq, q.nwg, q.n, q.d, q.w32, q.lambda, q.UT, q.lam, q.k, q.mu,
                                   q.tmp, q.state, q.stop_rule, q.eps, q.f_star, q.wt, q.wt_prev, first);
  if ((action == 1 || action == 2 || action == 3) && threadIdx.x == 0) {
    const int before = atomicAdd(done_count, 1);
    if (before + 1 == nprob && host_stop) __hip_atomic_store(host_stop, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// The P^{-1/2} apply of a single problem over several workgroups, for large k d: the same per-row and
// per-quad arithmetic as pmhalf_apply_block (so the results are bit-identical), with phase 1 on
// ceil(k / 4) one-wave workgroups and phase 2 on 256-thread workgroups of 64 column quads, so that
// U~^T streams through many CUs instead of one. tb (k doubles, global) carries the coefficients.
// Measured break-even of 14-epoch solves: one workgroup is 1-2 us per epoch faster at k d = 16384
// (d = 512, k = 32), the split 2.5 us faster at k d = 20000 (d = 1000, k = 20) and 7 us at 50000.
constexpr int64_t kSplitApplyMin = 20000;  // k d from which the split kernels are used

bool split_apply(const float* UT, int k, int64_t d) {
  return k > 0 && (d & 3) == 0 && (reinterpret_cast<uintptr_t>(UT) & 15) == 0 && (int64_t)k * d >= kSplitApplyMin;
}

template <typename VIN>
__global__ __launch_bounds__(64) void pmhalf_rows_kernel(const float* UT, const double* lam, int k, int64_t d,
                                                         double lambda, const VIN* v, double* tb,
                                                         const SolveState* state) {
  if (state && state->done) return;
  const double s = sqrt(fmax(lam[k - 1], 0.0) + lambda);
  pmhalf_rows_v4(UT, lam, k, d, lambda, s, (int)blockIdx.x * kApplyR, (int)threadIdx.x & 63,
                 [&](int j) { return (double)v[j]; }, tb);
}

// phase 2 of the premap: w = P^{-1/2} w~ (and the trace row)
__global__ __launch_bounds__(256) void premap_cols_kernel(const float* UT, const double* lam, int k, int64_t d,
                                                          double lambda, const float* wt, const double* tb, float* w,
                                                          float* trace_row, const SolveState* state) {
  if (state && state->done) return;
  const double s = sqrt(fmax(lam[k - 1], 0.0) + lambda);
  pmhalf_quad_v4(UT, tb, k, d, s, (int)blockIdx.x * 64 + ((int)threadIdx.x >> 2), (int)threadIdx.x & 3,
                 [&](int j) { return (double)wt[j]; }, [&](int j, double x) {
                   const float f = (float)x;
                   w[j] = f;
                   if (trace_row) trace_row[j] = f;
                 });
}

// gradient finish, step 1: g = (1/n) sum of the workgroup partial rows + lambda w, 64 columns per
// workgroup. Wave q forms row group q's sum exactly as colreduce_body does (four row slices, each
// added in row order, then ((s0 + s1) + s2) + s3), and wave 0 adds the kColSplit group sums in group
// order and finishes as grad_entry does: g is bit-identical to colreduce followed by grad_entry, in
// one launch instead of two.
__global__ __launch_bounds__(64 * kColSplit) void grad_colsum_kernel(const float* part, int nwg, int64_t n, int64_t d,
                                                                      const float* w, double lambda, double* g,
                                                                      const SolveState* state) {
  if (state && state->done) return;
  __shared__ double sg[kColSplit][64];
  const int c = threadIdx.x & 63, by = threadIdx.x >> 6;
  const int64_t j = (int64_t)blockIdx.x * 64 + c;
  const int R = (nwg + kColSplit - 1) / kColSplit;
  const int r0 = by * R, r1 = r0 + R < nwg ? r0 + R : nwg;
  double sl[4] = {0.0, 0.0, 0.0, 0.0};
  if (j < d) {
#pragma unroll
    for (int rs = 0; rs < 4; ++rs) {
#pragma unroll 4
      for (int q = r0 + rs; q < r1; q += 4) sl[rs] += (double)part[(int64_t)q * d + j];
    }
  }
  sg[by][c] = ((sl[0] + sl[1]) + sl[2]) + sl[3];
  __syncthreads();
  if (by == 0 && j < d) {
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < kColSplit; ++q) acc += sg[q][c];
    g[j] = acc / (double)n + lambda * (double)w[j];
  }
}

// step 3: mu = P^{-1/2} g into tmp
__global__ __launch_bounds__(256) void grad_mu_cols_kernel(const float* UT, const double* lam, int k, int64_t d,
                                                           double lambda, const double* g, const double* tb,
                                                           double* tmp, const SolveState* state) {
  if (state->done) return;
  const double s = sqrt(fmax(lam[k - 1], 0.0) + lambda);
  pmhalf_quad_v4(UT, tb, k, d, s, (int)blockIdx.x * 64 + ((int)threadIdx.x >> 2), (int)threadIdx.x & 3,
                 [&](int j) { return g[j]; }, [&](int j, double x) { tmp[j] = x; });
}

// step 4: the finish once tmp holds mu (one workgroup), with the host flag of grad_finalize_kernel
__global__ __launch_bounds__(kVecThreads) void grad_tail_kernel(
    const double* rsq_part, int nwg, int64_t n, int64_t d, const float* w, double lambda, const double* lam, int k,
    float* mu, const double* tmp, SolveState* state, int stop_rule, double eps, double f_star, float* wt_cur,
    const float* wt_prev, int first, int* host_stop) {
  if (state->done) {
    if (host_stop && threadIdx.x == 0) __hip_atomic_store(host_stop, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    return;
  }
  const int action = finalize_tail(rsq_part, nwg, n, d, w, lambda, lam, k, mu, tmp, state, stop_rule, eps, f_star,
                                   wt_cur, wt_prev, first);
  if (host_stop && threadIdx.x == 0)
    __hip_atomic_store(host_stop, (action == 1 || action == 2 || action == 3) ? 1 : 2, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_SYSTEM);
}

__global__ void rownorm_kernel(const float* X, int64_t n, int64_t d, int64_t ldx, float* out) {
  int64_t r = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  int lane = threadIdx.x & 63;
  if (r >= n) return;
  const float* p = X + r * ldx;
  float acc = 0.f;
  for (int64_t j = lane; j < d; j += 64) acc = fmaf(p[j], p[j], acc);
  acc = warp_sum(acc);
  if (lane == 0) out[r] = acc;
}

__global__ void rownorm_bf16_kernel(const uint16_t* X, int64_t n, int64_t d, float* out) {
  int64_t r = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  int lane = threadIdx.x & 63;
  if (r >= n) return;
  const uint16_t* p = X + r * d;
  float acc = 0.f;
  for (int64_t j = lane; j < d; j += 64) {
    float x = bf16_to_f32(p[j]);
    acc = fmaf(x, x, acc);
  }
  acc = warp_sum(acc);
  if (lane == 0) out[r] = acc;
}

__global__ void copy_bf16_kernel(const float* X, int64_t n, int64_t d, int64_t ldx, uint16_t* out) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * d) return;
  int64_t r = e / d, c = e - r * d;
  out[e] = f32_to_bf16(X[r * ldx + c]);
}

__global__ void fill_identity_kernel(int64_t d, float alpha, int bf16, void* out, float* beta_reg) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= d * d) return;
  int64_t r = e / d, c = e - r * d;
  float v = r == c ? alpha : 0.f;
  if (bf16) {
    uint16_t h = f32_to_bf16(v);
    reinterpret_cast<uint16_t*>(out)[e] = h;
    if (r == c && beta_reg) {
      float q = bf16_to_f32(h);
      beta_reg[r] = q * q;
    }
  } else {
    reinterpret_cast<float*>(out)[e] = v;
    if (r == c && beta_reg) beta_reg[r] = v * v;
  }
}

__global__ void transpose_kernel(const float* A, int64_t rows, int64_t cols, float* AT) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  int64_t r = e / cols, c = e - r * cols;
  AT[c * rows + r] = A[e];
}

// U~ = Q V_k with the columns of V taken in descending order of theta; lam = max(theta, 0).
__device__ __forceinline__ void lift_body(int64_t e, const double* Q, int64_t d, int l, const double* V,
                                          const int* order, int k, const double* theta, double* U64, float* U32,
                                          float* UT32, double* lam, float* VkT) {
  if (e < d * k) {
    int64_t j = e / k;
    int i = (int)(e - j * k);
    int col = order[i];
    double acc = 0.0;
    for (int c = 0; c < l; ++c) acc += Q[j * l + c] * V[(int64_t)c * l + col];
    if (U64) U64[j * k + i] = acc;
    U32[j * k + i] = (float)acc;
    UT32[(int64_t)i * d + j] = (float)acc;
  }
  if (e < (int64_t)k * l) {
    int i = (int)(e / l), c = (int)(e - (int64_t)i * l);
    VkT[e] = (float)V[(int64_t)c * l + order[i]];
  }
  if (e < k) lam[e] = fmax(theta[order[e]], 0.0);
}

__global__ void lift_kernel(const double* Q, int64_t d, int l, const double* V, const int* order, int k,
                            const double* theta, double* U64, float* U32, float* UT32, double* lam, float* VkT) {
  lift_body((int64_t)blockIdx.x * blockDim.x + threadIdx.x, Q, d, l, V, order, k, theta, U64, U32, UT32, lam, VkT);
}

// job blockIdx.y; its elements beyond max(d k, k l) are idle threads
__global__ void lift_batched_kernel(const LiftJob* jobs) {
  const LiftJob j = jobs[blockIdx.y];
  lift_body((int64_t)blockIdx.x * blockDim.x + threadIdx.x, j.Q, j.d, j.l, j.V, j.order, j.k, j.theta, j.U64,
            j.U32, j.UT32, j.lam, j.VkT);
}

// s = sqrt(lam_k + lambda); D_i = 1/sqrt(lam_i + lambda) - 1/s; UD = U diag(D) and Up = U, both with
// leading dimension ldu and zero past column k and past row d (up to drows rows);
// scal[0] = 1/s (row scale of the apply), scal[1] = sqrt(n lambda)/s (diagonal of the regularizer rows).
__global__ void precond_setup_kernel(const double* lam, int k, double lambda, int64_t n, const float* U32,
                                     int64_t d, int64_t drows, float* UD, float* Up, int64_t ldu, double* scal,
                                     SolveState* state) {
  double s = sqrt(fmax(lam[k - 1], 0.0) + lambda);
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < drows * ldu) {
    const int64_t r = e / ldu;
    const int i = (int)(e - r * ldu);
    float ud = 0.f, u = 0.f;
    if (r < d && i < k) {
      double D = 1.0 / sqrt(fmax(lam[i], 0.0) + lambda) - 1.0 / s;
      u = U32[r * k + i];
      ud = (float)((double)u * D);
    }
    UD[e] = ud;
    Up[e] = u;
  }
  if (e == 0) {
    scal[0] = 1.0 / s;
    scal[1] = sqrt((double)n * lambda) / s;
    if (state) {
      state->s = s;
      state->lam_top = fmax(lam[0], 0.0);
    }
  }
}

// Zeroes up to three buffers of 4-byte words in one launch (a, b, c may be null with count 0).
__global__ void zero3_kernel(uint32_t* a, int64_t na, uint32_t* b, int64_t nb, uint32_t* c, int64_t nc) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < na) a[e] = 0u;
  if (e < nb) b[e] = 0u;
  if (e < nc) c[e] = 0u;
}

}  // namespace

int launch_zero3(hipStream_t st, void* a, int64_t abytes, void* b, int64_t bbytes, void* c, int64_t cbytes) {
  if ((abytes | bbytes | cbytes) & 3) {
    set_error("zero3: sizes must be multiples of 4 bytes");
    return SCS_EINVAL;
  }
  const int64_t na = a ? abytes / 4 : 0, nb = b ? bbytes / 4 : 0, nc = c ? cbytes / 4 : 0;
  const int64_t mx = std::max(na, std::max(nb, nc));
  if (mx == 0) return SCS_OK;
  zero3_kernel<<<(unsigned)cdiv(mx, 256), 256, 0, st>>>(reinterpret_cast<uint32_t*>(a), na,
                                                         reinterpret_cast<uint32_t*>(b), nb,
                                                         reinterpret_cast<uint32_t*>(c), nc);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_premap(hipStream_t st, const float* UT, const float* U, const double* lam, int k, int64_t d,
                  double lambda, const float* wt, float* w, float* trace_row, double* tmp,
                  const SolveState* state) {
  (void)U;
  if (split_apply(UT, k, d)) {  // tmp (d >= k doubles) carries the coefficients between the two phases
    pmhalf_rows_kernel<float><<<(unsigned)cdiv(k, kApplyR), 64, 0, st>>>(UT, lam, k, d, lambda, wt, tmp, state);
    SCS_HIP(hipGetLastError());
    premap_cols_kernel<<<(unsigned)cdiv(d >> 2, 64), 256, 0, st>>>(UT, lam, k, d, lambda, wt, tmp, w, trace_row,
                                                                    state);
    SCS_HIP(hipGetLastError());
    return SCS_OK;
  }
  premap_kernel<<<1, kVecThreads, 0, st>>>(UT, lam, k, d, lambda, wt, w, trace_row, tmp, state);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_grad_finish(hipStream_t st, const float* part, const double* rsq_part, int nwg, int64_t n, int64_t d,
                       const float* w, double lambda, const float* UT, const float* U, const double* lam, int k,
                       float* mu, double* g_tmp, double* tmp, SolveState* state, int stop_rule, double eps,
                       double f_star, float* wt_cur, const float* wt_prev, int first, int* host_stop) {
  (void)U;
  if (split_apply(UT, k, d)) {  // g over row 0 of g_tmp, the coefficients in row 1, mu in tmp
    grad_colsum_kernel<<<(unsigned)cdiv(d, 64), 64 * kColSplit, 0, st>>>(part, nwg, n, d, w, lambda, g_tmp, state);
    SCS_HIP(hipGetLastError());
    pmhalf_rows_kernel<double><<<(unsigned)cdiv(k, kApplyR), 64, 0, st>>>(UT, lam, k, d, lambda, g_tmp, g_tmp + d,
                                                                         state);
    SCS_HIP(hipGetLastError());
    grad_mu_cols_kernel<<<(unsigned)cdiv(d >> 2, 64), 256, 0, st>>>(UT, lam, k, d, lambda, g_tmp, g_tmp + d, tmp,
                                                                     state);
    SCS_HIP(hipGetLastError());
    grad_tail_kernel<<<1, kVecThreads, 0, st>>>(rsq_part, nwg, n, d, w, lambda, lam, k, mu, tmp, state, stop_rule,
                                                eps, f_star, wt_cur, wt_prev, first, host_stop);
    SCS_HIP(hipGetLastError());
    return SCS_OK;
  }
  grad_colreduce_kernel<<<dim3((unsigned)cdiv(d, 64), kColSplit), dim3(256), 0, st>>>(part, nwg, d, g_tmp, state);
  SCS_HIP(hipGetLastError());
  grad_finalize_kernel<<<1, kVecThreads, 0, st>>>(g_tmp, rsq_part, nwg, n, d, w, lambda, UT, lam, k, mu, tmp,
                                                  state, stop_rule, eps, f_star, wt_cur, wt_prev, first, host_stop);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

// Sec. 2.2: out[0] = (k lam_k + tail)/(n k) (Eq. (decay)), out[1] = tr(C)/(n k) (Eq. (decaySVRG)), with
// tr(C) = sum_i ||x_i||^2 / n from the sampler's FP64 sum of the row norms and tail = tr(C) - sum of the
// k sketched eigenvalues (clamped at 0).
__global__ void budget_lambda_kernel(const double* lam, int k, const SolveState* state, int64_t n, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double trace = state->beta_sum / (double)n;
  double top = 0.0;
  for (int i = 0; i < k; ++i) top += fmax(lam[i], 0.0);
  const double tail = fmax(trace - top, 0.0);
  const double nk = (double)n * (double)k;
  out[0] = ((double)k * fmax(lam[k - 1], 0.0) + tail) / nk;
  out[1] = trace / nk;
}

int launch_budget_lambda(hipStream_t st, const double* lam, int k, const SolveState* state, int64_t n, double* out) {
  budget_lambda_kernel<<<1, 64, 0, st>>>(lam, k, state, n, out);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_pmhalf_inv(hipStream_t st, const float* UT, const double* lam, int k, int64_t d, double lambda,
                      const float* w, float* wt) {
  if (k > kMaxPmhalfInvK) {
    set_error("P^{1/2} map: k too large");
    return SCS_EINVAL;
  }
  pmhalf_inv_kernel<<<1, 256, 0, st>>>(UT, lam, k, d, lambda, w, wt);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_premap_batched(hipStream_t st, const BatchProb* P, int nprob, int final_out, float* const* w_out) {
  if (nprob < 1) return SCS_OK;
  premap_batched_kernel<<<nprob, kVecThreads, 0, st>>>(P, final_out, w_out);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_grad_finish_batched(hipStream_t st, const BatchProb* P, int nprob, const int64_t* cb_prefix,
                               int64_t total_cb, int first, int* done_count, int* host_stop, const int* clk) {
  if (nprob < 1) return SCS_OK;
  grad_colreduce_batched_kernel<<<dim3((unsigned)total_cb, kColSplit), dim3(256), 0, st>>>(P, nprob, cb_prefix);
  SCS_HIP(hipGetLastError());
  return launch_grad_finalize_batched(st, P, nprob, first, done_count, host_stop, clk);
}

int launch_grad_finalize_batched(hipStream_t st, const BatchProb* P, int nprob, int first, int* done_count,
                                 int* host_stop, const int* clk) {
  if (nprob < 1) return SCS_OK;
  grad_finalize_batched_kernel<<<nprob, kVecThreads, 0, st>>>(P, nprob, first, done_count, host_stop, clk);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

__global__ void clock_set_kernel(int* clk, int epoch, int epochs) {
  if (threadIdx.x == 0) {
    clk[0] = epoch;
    clk[1] = epochs;
  }
}

__global__ void clock_advance_kernel(int* clk) {
  if (threadIdx.x == 0 && clk[0] <= clk[1]) clk[0] += 1;
}

int launch_clock_set(hipStream_t st, int* clk, int epoch, int epochs) {
  clock_set_kernel<<<1, 64, 0, st>>>(clk, epoch, epochs);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_clock_advance(hipStream_t st, int* clk) {
  clock_advance_kernel<<<1, 64, 0, st>>>(clk);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_rownorm(hipStream_t st, const float* X, int64_t n, int64_t d, int64_t ldx, float* out) {
  if (n <= 0) return SCS_OK;
  rownorm_kernel<<<dim3((unsigned)cdiv(n, 4)), dim3(256), 0, st>>>(X, n, d, ldx, out);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_rownorm_bf16(hipStream_t st, const uint16_t* X, int64_t n, int64_t d, float* out) {
  if (n <= 0) return SCS_OK;
  rownorm_bf16_kernel<<<dim3((unsigned)cdiv(n, 4)), dim3(256), 0, st>>>(X, n, d, out);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_copy_bf16(hipStream_t st, const float* X, int64_t n, int64_t d, int64_t ldx, uint16_t* out) {
  if (n * d <= 0) return SCS_OK;
  copy_bf16_kernel<<<dim3((unsigned)cdiv(n * d, 256)), dim3(256), 0, st>>>(X, n, d, ldx, out);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_transpose_f32(hipStream_t st, const float* A, int64_t rows, int64_t cols, float* AT) {
  if (rows * cols <= 0) return SCS_OK;
  transpose_kernel<<<dim3((unsigned)cdiv(rows * cols, 256)), dim3(256), 0, st>>>(A, rows, cols, AT);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_fill_scaled_identity(hipStream_t st, int64_t d, double alpha, int bf16, void* out, float* beta_reg) {
  fill_identity_kernel<<<dim3((unsigned)cdiv(d * d, 256)), dim3(256), 0, st>>>(d, (float)alpha, bf16, out,
                                                                               beta_reg);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_lift(hipStream_t st, const double* Q, int64_t d, int l, const double* V, const int* order, int k,
                const double* theta, double* U64, float* U32, float* UT32, double* lam, float* VkT) {
  int64_t tot = d * k > (int64_t)k * l ? d * k : (int64_t)k * l;
  lift_kernel<<<dim3((unsigned)cdiv(tot, 256)), dim3(256), 0, st>>>(Q, d, l, V, order, k, theta, U64, U32, UT32,
                                                                    lam, VkT);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_lift_batched(hipStream_t st, const LiftJob* jobs, int njobs, int64_t max_elems) {
  if (njobs <= 0 || max_elems <= 0) return SCS_OK;
  lift_batched_kernel<<<dim3((unsigned)cdiv(max_elems, 256), (unsigned)njobs), dim3(256), 0, st>>>(jobs);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_precond_setup(hipStream_t st, const double* lam, int k, double lambda, int64_t n, const float* U32,
                         int64_t d, float* UD, float* Up, int64_t ldu, double* scal, SolveState* state) {
  const int64_t drows = gemm_wide_bt_rows(d);
  precond_setup_kernel<<<dim3((unsigned)cdiv(drows * ldu, 256)), dim3(256), 0, st>>>(lam, k, lambda, n, U32, d, drows,
                                                                                     UD, Up, ldu, scal, state);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

}  // namespace scs
