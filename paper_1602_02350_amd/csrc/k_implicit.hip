// SVRG inner loop with the sketched preconditioner applied implicitly (Eq. (condSketch)): the rows
// x~_i = x_i / s + U~ D z_i (z_i = U~^T x_i, D_r = 1/sqrt(lam~_r + lambda) - 1/s) are never formed.
// The correction delta = w~_t - w~ of Alg. 1 is kept as delta_x + U~ delta_a (delta_x in R^d,
// delta_a in R^k) together with c = U~^T delta_x. With U~^T U~ = I,
//   x~_i^T delta = x_i^T delta_x / s + z_i^T v,          v = delta_a / s + D (c + delta_a),
// and the step delta -= eta (sum_j g_j x~_{i_j} + mu) splits into
//   delta_x -= eta (sum_j g_j x_{i_j} / s + mu),  c -= eta (sum_j g_j z_{i_j} / s + U~^T mu),
//   delta_a -= eta D sum_j g_j z_{i_j},
// O(d + k) per sampled row. A regularizer row i = n + j is sqrt(n lambda) P^{-1/2} e_j: its x-part
// is sqrt(n lambda) e_j and its z-part sqrt(n lambda) times row j of U~. The snapshot becomes
// w~ + avg(delta_x) + U~ avg(delta_a). Rows of X and Z are shared by every lambda of a path.
//
// One workgroup per problem (no cross-workgroup exchange): waves take sampled rows and reduce
// each row's dot product inside the wave; threads then own columns (and components of the
// k-vectors) for the update, re-reading the step's rows from cache.
#include "scs_internal.h"

namespace scs {

namespace {

constexpr int kImpThreads = 512;
constexpr int kImpWaves = kImpThreads / 64;
constexpr int kImpMaxD = 2048;
constexpr int kImpMaxK = 128;

__device__ __forceinline__ float wave_sum_f_fast(float v) {
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x128, 0xf, 0xf, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x124, 0xf, 0xf, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x122, 0xf, 0xf, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x121, 0xf, 0xf, false));
  auto p16 = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  v = __uint_as_float(p16[0]) + __uint_as_float(p16[1]);
  auto p32 = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(p32[0]) + __uint_as_float(p32[1]);
}

__global__ __launch_bounds__(kImpThreads) void inner_implicit_kernel(const BatchProb* P, int slot, int64_t epoch,
                                                                     const int* clk) {
  if (clk) {  // epochs replayed from a graph: the epoch number is on the device
    if (clk[0] >= clk[1]) return;
    slot = clk[0] % kEpochGroup;
  }
  const BatchProb& q = P[blockIdx.x];
  if (q.state->done) return;
  const InnerArgs& a = q.inner;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t n = q.n;
  const int d = (int)q.d, k = q.k, b = a.b;
  const int64_t m = a.m, ldx = a.ldx;
  const float* X = reinterpret_cast<const float*>(a.Xt);
  const float* Z = q.Z;
  const float* UT = q.UT;
  const int32_t* idx = q.idx + (int64_t)slot * q.draws;
  const float* scl = q.scale + (int64_t)slot * q.draws;
  (void)epoch;

  __shared__ float dx[kImpMaxD], sx[kImpMaxD], cx[kImpMaxD], mux[kImpMaxD];
  __shared__ float da[kImpMaxK], sa[kImpMaxK], ka[kImpMaxK], cc[kImpMaxK], Ds[kImpMaxK], muz[kImpMaxK], vv[kImpMaxK];
  __shared__ float gam[64];
  __shared__ int sidx[64];

  const double lam_k = k > 0 ? fmax(q.lam[k - 1], 0.0) : 0.0;
  const double s = sqrt(lam_k + q.lambda);
  const float is = (float)(1.0 / s);
  const float sq = (float)sqrt((double)n * q.lambda);
  const float eta = (float)ldexp(a.step_scale * (double)n / q.state->beta_sum, -q.state->backoffs);

  for (int c = tid; c < d; c += kImpThreads) {
    dx[c] = 0.f;
    sx[c] = 0.f;
    cx[c] = 0.f;
    mux[c] = a.mu[c];
  }
  for (int r = tid; r < k; r += kImpThreads) {
    da[r] = 0.f;
    sa[r] = 0.f;
    ka[r] = 0.f;
    cc[r] = 0.f;
    vv[r] = 0.f;
    Ds[r] = (float)(1.0 / sqrt(fmax(q.lam[r], 0.0) + q.lambda) - 1.0 / s);
  }
  // U~^T mu, one wave per component
  for (int r = wave; r < k; r += kImpWaves) {
    float acc = 0.f;
    for (int c = lane; c < d; c += 64) acc = fmaf(UT[(int64_t)r * d + c], a.mu[c], acc);
    acc = wave_sum_f_fast(acc);
    if (lane == 0) muz[r] = acc;
  }
  __syncthreads();

  for (int64_t t = 0; t < m; ++t) {
    if (tid < b) sidx[tid] = idx[t * b + tid];
    __syncthreads();
    // dot products of the sampled rows with the current correction, one wave per row
    for (int j = wave; j < b; j += kImpWaves) {
      const uint32_t i = (uint32_t)sidx[j];
      float p = 0.f;
      if (i < (uint32_t)n) {
        const float* row = X + (int64_t)i * ldx;
        for (int c = 4 * lane; c < d; c += 256) {
          const float4 x4 = *reinterpret_cast<const float4*>(row + c);
          p = fmaf(x4.x, dx[c], p);
          if (c + 1 < d) p = fmaf(x4.y, dx[c + 1], p);
          if (c + 2 < d) p = fmaf(x4.z, dx[c + 2], p);
          if (c + 3 < d) p = fmaf(x4.w, dx[c + 3], p);
        }
        p *= is;
        const float* zr = Z + (int64_t)i * q.ldz;
        for (int r = lane; r < k; r += 64) p = fmaf(zr[r], vv[r], p);
      } else {
        const int jj = (int)(i - (uint32_t)n);
        if (lane == 0) p = dx[jj] * is;
        for (int r = lane; r < k; r += 64) p = fmaf(UT[(int64_t)r * d + jj], vv[r], p);
        p *= sq;
      }
      p = wave_sum_f_fast(p);
      if (lane == 0) gam[j] = p * scl[t * b + j] / (float)b;
    }
    __syncthreads();
    // delta_x: columns owned by threads, the step's rows re-read from cache
    for (int c = tid; c < d; c += kImpThreads) {
      float g = 0.f;
      for (int j = 0; j < b; ++j) {
        const uint32_t i = (uint32_t)sidx[j];
        if (i < (uint32_t)n) g = fmaf(gam[j], X[(int64_t)i * ldx + c], g);
        else if ((int)(i - (uint32_t)n) == c) g = fmaf(gam[j], sq, g);
      }
      const float nd = dx[c] - eta * (is * g + mux[c]);
      dx[c] = nd;
      const float y = nd - cx[c];
      const float s2 = sx[c] + y;
      cx[c] = (s2 - sx[c]) - y;
      sx[c] = s2;
    }
    // delta_a and c: components owned by threads
    for (int r = tid; r < k; r += kImpThreads) {
      float gz = 0.f;
      for (int j = 0; j < b; ++j) {
        const uint32_t i = (uint32_t)sidx[j];
        const float zv = i < (uint32_t)n ? Z[(int64_t)i * q.ldz + r] : sq * UT[(int64_t)r * d + (int)(i - (uint32_t)n)];
        gz = fmaf(gam[j], zv, gz);
      }
      const float nda = da[r] - eta * Ds[r] * gz;
      const float ncc = cc[r] - eta * (is * gz + muz[r]);
      da[r] = nda;
      cc[r] = ncc;
      const float y = nda - ka[r];
      const float s2 = sa[r] + y;
      ka[r] = (s2 - sa[r]) - y;
      sa[r] = s2;
      vv[r] = nda * is + Ds[r] * (ncc + nda);
    }
    __syncthreads();
  }
  // snapshot: w~ + avg(delta_x) + U~ avg(delta_a) (or the last correction)
  const float inv_m = 1.0f / (float)m;
  for (int c = tid; c < d; c += kImpThreads) {
    float u = a.average ? (sx[c] - cx[c]) * inv_m : dx[c];
    for (int r = 0; r < k; ++r) {
      const float ar = a.average ? (sa[r] - ka[r]) * inv_m : da[r];
      u = fmaf(UT[(int64_t)r * d + c], ar, u);
    }
    const float w0 = a.wt[c];
    if (a.wt_prev) a.wt_prev[c] = w0;
    a.wt[c] = w0 + u;
  }
  if (tid == 0) {
    q.state->epochs += 1;
    q.state->eta = (double)eta;
  }
}

// beta_i = ||x~_i||^2 = ||x_i||^2 / s^2 + z_i^T (2 D / s + D^2) z_i for data rows and
// n lambda (1/s^2 + u_j^T (2 D / s + D^2) u_j) for regularizer rows, without forming x~.
__global__ void implicit_beta_kernel(const float* xnorm2, const float* Z, int64_t ldz, const float* UT,
                                     const double* lam, int k, int64_t n, int64_t d, double lambda, float* beta) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n + d) return;
  const double s = sqrt(fmax(k > 0 ? lam[k - 1] : 0.0, 0.0) + lambda);
  double acc = 0.0;
  for (int r = 0; r < k; ++r) {
    const double D = 1.0 / sqrt(fmax(lam[r], 0.0) + lambda) - 1.0 / s;
    const double z = i < n ? (double)Z[i * ldz + r] : (double)UT[(int64_t)r * d + (i - n)];
    acc += z * z * (2.0 * D / s + D * D);
  }
  beta[i] = i < n ? (float)((double)xnorm2[i] / (s * s) + acc) : (float)((double)n * lambda * (1.0 / (s * s) + acc));
}

}  // namespace

int launch_inner_implicit_batched(hipStream_t st, const BatchProb* P, int nprob, int64_t max_d, int max_k, int max_b,
                                  int epoch_slot, int64_t epoch, const int* clk) {
  if (nprob < 1) return SCS_OK;
  if (max_d > kImpMaxD || max_k > kImpMaxK || max_b > 64) {
    set_error("implicit inner loop: needs d <= 2048, k <= 128, b <= 64");
    return SCS_EINVAL;
  }
  inner_implicit_kernel<<<nprob, kImpThreads, 0, st>>>(P, epoch_slot, epoch, clk);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_implicit_beta(hipStream_t st, const float* xnorm2, const float* Z, int64_t ldz, const float* UT,
                         const double* lam, int k, int64_t n, int64_t d, double lambda, float* beta) {
  implicit_beta_kernel<<<dim3((unsigned)cdiv(n + d, 256)), dim3(256), 0, st>>>(xnorm2, Z, ldz, UT, lam, k, n, d,
                                                                               lambda, beta);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

}  // namespace scs
