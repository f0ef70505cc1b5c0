// FP64 dense algebra on the small matrices of the sketch (l = k + p <= 136):
//  * gemm64: C = A B with arbitrary strides (covers transposes), 16x16 LDS tiles;
//  * chol_inv64: G = R^T R (upper R) and R^{-1}, one workgroup, packed triangles, for CholeskyQR2
//    (Q = Y R^{-1}, twice; Fukaya, Nakatsukasa, Yanagisawa, Yamamoto 2014);
//  * jacobi64: symmetric eigendecomposition B = V diag(theta) V^T by cyclic Jacobi with the
//    round-robin parallel ordering (l/2 disjoint rotations per round), one workgroup; the
//    eigenvalues are returned with their descending order (Rayleigh-Ritz step of Alg. 2).
#include "scs_internal.h"

namespace scs {

namespace {

constexpr int kT = 16;

// 16x16 output tile per workgroup; the K range is split over kKZ thread slices (threadIdx.z) that
// walk interleaved 16-wide K tiles in lockstep, and their partial tiles are added in slice order.
constexpr int kKZ = 4;

__global__ __launch_bounds__(kT * kT * kKZ) void gemm64_kernel(int64_t M, int64_t N, int64_t K, const double* A,
                                                               int64_t a_rs, int64_t a_cs, const double* B,
                                                               int64_t b_rs, int64_t b_cs, double* C, int64_t ldc,
                                                               float* C32, int64_t ldc32) {
  __shared__ double As[kKZ][kT][kT + 1], Bs[kKZ][kT][kT + 1];
  const int tx = threadIdx.x, ty = threadIdx.y, tz = threadIdx.z;
  const int64_t i = (int64_t)blockIdx.y * kT + ty, j = (int64_t)blockIdx.x * kT + tx;
  double acc = 0.0;
  const int64_t iters = (K + kT * kKZ - 1) / (kT * kKZ);
  for (int64_t it = 0; it < iters; ++it) {
    const int64_t k0 = (it * kKZ + tz) * kT;
    int64_t ka = k0 + tx, kb = k0 + ty;
    As[tz][ty][tx] = (i < M && ka < K) ? A[i * a_rs + ka * a_cs] : 0.0;
    Bs[tz][ty][tx] = (kb < K && j < N) ? B[kb * b_rs + j * b_cs] : 0.0;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kT; ++q) acc += As[tz][ty][q] * Bs[tz][q][tx];
    __syncthreads();
  }
  As[tz][ty][tx] = acc;
  __syncthreads();
  if (tz == 0 && i < M && j < N) {
    double v = As[0][ty][tx];
#pragma unroll
    for (int z = 1; z < kKZ; ++z) v += As[z][ty][tx];
    if (C) C[i * ldc + j] = v;
    if (C32) C32[i * ldc32 + j] = (float)v;
  }
}

// Cholesky G = R^T R (upper R) and R^{-1}, one workgroup, R packed in LDS (l (l + 1) / 2 doubles).
// Right-looking with one barrier per column: phase j reads the finished diagonal entry p_j and the
// unscaled row j, updates the trailing triangle with S[a][c] -= S[j][a] S[j][c] / p_j, and scales
// row j - 1 (which nothing reads in that phase) by 1/sqrt(p_{j-1}). The inverse X = R^{-1} is then
// formed one column per wave by back substitution in axpy form: x = e_j, and for q = j, ..., 0:
// x_q /= R[q][q], x_i -= R[i][q] x_q (i < q); lane t keeps x_t, x_{t+64}, x_{t+128} in registers.
// flag: 0 on success, 1 if a pivot is not positive relative to the largest diagonal entry of G
// (that pivot is replaced by 1 so the factor stays finite).
constexpr int kCholThreads = 512;

__device__ __forceinline__ int packed_up(int i, int j, int l) { return i * (2 * l - i + 1) / 2 + (j - i); }

__device__ __forceinline__ double readlane_d(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__global__ __launch_bounds__(kCholThreads) void chol_inv64_kernel(const double* G, int l, double* Rinv, int* flag) {
  extern __shared__ double S[];
  __shared__ double s_dmax;
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = tid >> 6, nwave = nt >> 6;
  for (int e = tid; e < l * l; e += nt) {
    int i = e / l, j = e % l;
    if (j >= i) S[packed_up(i, j, l)] = G[e];
  }
  if (tid == 0) {
    double m = 0.0;
    for (int j = 0; j < l; ++j) m = fmax(m, fabs(G[j * l + j]));
    s_dmax = m;
  }
  __syncthreads();
  const double dmax = s_dmax;
  int bad = 0;
  double p_prev = 1.0;
  auto pivot = [&](int j) {
    double p = S[packed_up(j, j, l)];
    if (!(p > 1e-30 * dmax) || !isfinite(p)) {
      bad = 1;
      p = 1.0;
    }
    return p;
  };
  auto finish_row = [&](int r, double p) {
    const double sp = sqrt(p), isp = 1.0 / sp;
    for (int c = r + tid; c < l; c += nt) S[packed_up(r, c, l)] = c == r ? sp : S[packed_up(r, c, l)] * isp;
  };
  for (int j = 0; j < l; ++j) {
    const double p = pivot(j), ip = 1.0 / p;
    const int m = l - j - 1;
    for (int e = tid; e < m * m; e += nt) {
      int a = j + 1 + e / m, c = j + 1 + e % m;
      if (c >= a) S[packed_up(a, c, l)] -= S[packed_up(j, a, l)] * S[packed_up(j, c, l)] * ip;
    }
    if (j > 0) finish_row(j - 1, p_prev);
    p_prev = p;
    __syncthreads();
  }
  finish_row(l - 1, p_prev);
  __syncthreads();
  for (int j = wave; j < l; j += nwave) {
    double x[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) x[r] = (lane + 64 * r == j) ? 1.0 : 0.0;
    for (int q = j; q >= 0; --q) {
      const int slot = q >> 6, owner = q & 63;  // uniform across the wave
      const double mine = slot == 0 ? x[0] : (slot == 1 ? x[1] : x[2]);
      const double xq = readlane_d(mine, owner) / S[packed_up(q, q, l)];
      if (lane == owner) {
        if (slot == 0) x[0] = xq;
        else if (slot == 1) x[1] = xq;
        else x[2] = xq;
      }
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const int i = lane + 64 * r;
        if (i < q) x[r] -= S[packed_up(i, q, l)] * xq;
      }
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const int i = lane + 64 * r;
      if (i < l) Rinv[(int64_t)i * l + j] = i <= j ? x[r] : 0.0;
    }
  }
  if (tid == 0) *flag = bad;
}

// Round-robin pairing: P players (P even), round t, slot s in [0, P/2): (pos s, pos P-1-s),
// player at position 0 is 0, at position q >= 1 it is 1 + (q - 1 + t) mod (P - 1).
__device__ __forceinline__ int rr_player(int pos, int t, int P) { return pos == 0 ? 0 : 1 + (pos - 1 + t) % (P - 1); }

// IN_LDS: the working matrix lives in LDS; V_LDS: the accumulated rotations too (copied to Vout at
// the end). Whatever does not fit stays in global memory (L2-resident at these sizes).
template <bool IN_LDS, bool V_LDS>
__global__ __launch_bounds__(1024) void jacobi64_kernel(const double* B, int l, double* Aglob, double* Vout,
                                                        double* theta, int* order, int max_sweeps) {
  extern __shared__ double S[];
  double* A = IN_LDS ? S : Aglob;
  double* V = V_LDS ? S + (IN_LDS ? l * l : 0) : Vout;
  __shared__ double cs_c[128], cs_s[128];
  __shared__ int cs_p[128], cs_q[128];
  __shared__ double s_tot;
  __shared__ int s_rot[2];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6, nwave = nt >> 6;
  if (tid == 0) s_tot = 0.0;
  __syncthreads();
  {
    double tot = 0.0;
    for (int e = tid; e < l * l; e += nt) {
      double a = B[e];
      A[e] = a;
      V[e] = (e / l == e % l) ? 1.0 : 0.0;
      tot += a * a;
    }
    tot = warp_sum_d(tot);
    if ((tid & 63) == 0) atomicAdd(&s_tot, tot);
  }
  __syncthreads();
  // A rotation is skipped when |a_pq| is below 1e-13 ||B||_F or below 1e-15 sqrt(|a_pp a_qq|) (the
  // off-diagonal rounding noise that rotations themselves leave is a few ulps of ||B||, so a floor at
  // the ulp level would never be met); a sweep without any rotation ends the iteration.
  const double abs_floor = 1e-13 * sqrt(s_tot);
  const int P = (l + 1) & ~1;
  const int half = P / 2;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    if (tid == 0) s_rot[sweep & 1] = 0;
    __syncthreads();
    for (int t = 0; t < P - 1; ++t) {
      for (int s = tid; s < half; s += nt) {
        int p = rr_player(s, t, P), q = rr_player(P - 1 - s, t, P);
        if (p > q) {
          int tmp = p;
          p = q;
          q = tmp;
        }
        double c = 1.0, sn = 0.0;
        if (q < l) {
          double apq = A[p * l + q];
          double app = A[p * l + p], aqq = A[q * l + q];
          if (fabs(apq) > abs_floor && fabs(apq) > 1e-15 * sqrt(fabs(app * aqq))) {
            s_rot[sweep & 1] = 1;
            double tau = (aqq - app) / (2.0 * apq);
            double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tt * tt);
            sn = tt * c;
          }
        } else {
          q = -1;  // the slot paired with the phantom index of an odd l: p is idle this round
        }
        cs_p[s] = p;
        cs_q[s] = q;
        cs_c[s] = c;
        cs_s[s] = sn;
      }
      __syncthreads();
      // The rotations of a round are disjoint, so A' = J^T A J is applied block by block in place:
      // the block of rows {p1, q1} and columns {p2, q2} depends only on itself (an idle slot
      // contributes one row or column with the identity). Slot pairs are spread over waves (s1) and
      // lanes (s2), so no index needs a division.
      for (int s1 = wave; s1 < half; s1 += nwave) {
        const int p1 = cs_p[s1], q1 = cs_q[s1];
        const double c1 = cs_c[s1], n1 = cs_s[s1];
        for (int s2 = lane; s2 < half; s2 += 64) {
          const int p2 = cs_p[s2], q2 = cs_q[s2];
          const double c2 = cs_c[s2], n2 = cs_s[s2];
          if (n1 == 0.0 && n2 == 0.0) continue;
          if (q1 >= 0 && q2 >= 0) {
            const double a_pp = A[p1 * l + p2], a_pq = A[p1 * l + q2];
            const double a_qp = A[q1 * l + p2], a_qq = A[q1 * l + q2];
            // rows: r_p = c1 r_p - n1 r_q, r_q = n1 r_p + c1 r_q; then the same on columns with (c2, n2)
            const double b_pp = c1 * a_pp - n1 * a_qp, b_pq = c1 * a_pq - n1 * a_qq;
            const double b_qp = n1 * a_pp + c1 * a_qp, b_qq = n1 * a_pq + c1 * a_qq;
            A[p1 * l + p2] = c2 * b_pp - n2 * b_pq;
            A[p1 * l + q2] = n2 * b_pp + c2 * b_pq;
            A[q1 * l + p2] = c2 * b_qp - n2 * b_qq;
            A[q1 * l + q2] = n2 * b_qp + c2 * b_qq;
          } else if (q1 >= 0) {  // column p2 is idle: row rotation only
            const double a_p = A[p1 * l + p2], a_q = A[q1 * l + p2];
            A[p1 * l + p2] = c1 * a_p - n1 * a_q;
            A[q1 * l + p2] = n1 * a_p + c1 * a_q;
          } else if (q2 >= 0) {  // row p1 is idle: column rotation only
            const double a_p = A[p1 * l + p2], a_q = A[p1 * l + q2];
            A[p1 * l + p2] = c2 * a_p - n2 * a_q;
            A[p1 * l + q2] = n2 * a_p + c2 * a_q;
          }
        }
      }
      for (int s = wave; s < half; s += nwave) {
        const int p = cs_p[s], q = cs_q[s];
        const double c = cs_c[s], sn = cs_s[s];
        if (q < 0 || sn == 0.0) continue;
        for (int i = lane; i < l; i += 64) {
          double vp = V[i * l + p], vq = V[i * l + q];
          V[i * l + p] = c * vp - sn * vq;
          V[i * l + q] = sn * vp + c * vq;
        }
      }
      __syncthreads();
    }
    if (s_rot[sweep & 1] == 0) break;
  }
  for (int i = tid; i < l; i += nt) theta[i] = A[i * l + i];
  if constexpr (V_LDS)
    for (int e = tid; e < l * l; e += nt) Vout[e] = V[e];
  __syncthreads();
  // rank sort, descending, ties by index
  for (int i = tid; i < l; i += nt) {
    double ti = A[i * l + i];
    int rank = 0;
    for (int j = 0; j < l; ++j) {
      double tj = A[j * l + j];
      if (tj > ti || (tj == ti && j < i)) ++rank;
    }
    order[rank] = i;
  }
}

int g_max_lds = -1;

int max_lds_bytes() {
  if (g_max_lds < 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return 65536;
    g_max_lds = (int)prop.sharedMemPerBlock;
  }
  return g_max_lds;
}

}  // namespace

int launch_gemm64(hipStream_t st, int64_t M, int64_t N, int64_t K, const double* A, int64_t a_rs, int64_t a_cs,
                  const double* B, int64_t b_rs, int64_t b_cs, double* C, int64_t ldc, float* C32,
                  int64_t ldc32) {
  if (M <= 0 || N <= 0) return SCS_OK;
  dim3 grid((unsigned)cdiv(N, kT), (unsigned)cdiv(M, kT));
  gemm64_kernel<<<grid, dim3(kT, kT, kKZ), 0, st>>>(M, N, K, A, a_rs, a_cs, B, b_rs, b_cs, C, ldc, C32, ldc32);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_chol_inv64(hipStream_t st, const double* G, int l, double* Rinv, int* flag) {
  const size_t bytes = (size_t)l * (l + 1) / 2 * sizeof(double);
  if (l > 192 || (int64_t)bytes + 1024 > max_lds_bytes()) {
    set_error("CholeskyQR: the sketch width k + p is too large for one workgroup");
    return SCS_EINVAL;
  }
  if (bytes > 65536) SCS_HIP(hipFuncSetAttribute((const void*)chol_inv64_kernel,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  chol_inv64_kernel<<<1, kCholThreads, bytes, st>>>(G, l, Rinv, flag);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_jacobi64(hipStream_t st, const double* B, int l, double* Awork, double* V, double* theta, int* order) {
  if (l > 256) {
    set_error("Jacobi: the sketch width k + p is too large");
    return SCS_EINVAL;
  }
  const size_t bytes = (size_t)l * l * sizeof(double);
  const int sweeps = 40;
  const int64_t room = max_lds_bytes() - 8192;  // static LDS of the kernel stays below 8 KB
  auto run = [&](auto kern, size_t dyn) -> int {
    if (dyn > 65536) SCS_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn));
    kern<<<1, 1024, dyn, st>>>(B, l, Awork, V, theta, order, sweeps);
    return SCS_OK;
  };
  if ((int64_t)(2 * bytes) <= room) {
    SCS_CHECK(run(jacobi64_kernel<true, true>, 2 * bytes));
  } else if ((int64_t)bytes <= room) {
    SCS_CHECK(run(jacobi64_kernel<true, false>, bytes));
  } else {
    SCS_CHECK(run(jacobi64_kernel<false, false>, 0));
  }
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

}  // namespace scs
