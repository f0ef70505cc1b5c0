// FP64 dense algebra on the small matrices of the sketch (l = k + p <= 136):
//  * gemm64: C = A B with arbitrary strides (covers transposes), 16x16 LDS tiles;
//  * chol_inv64: G = R^T R (upper R) and R^{-1}, one workgroup, for CholeskyQR2
//    (Q = Y R^{-1}, twice; Fukaya, Nakatsukasa, Yanagisawa, Yamamoto 2014);
//  * jacobi64: symmetric eigendecomposition B = V diag(theta) V^T by cyclic Jacobi with the
//    round-robin parallel ordering (l/2 disjoint rotations per round), one workgroup; the
//    eigenvalues are returned with their descending order (Rayleigh-Ritz step of Alg. 2).
#include "scs_internal.h"

namespace scs {

namespace {

constexpr int kT = 16;

__global__ void gemm64_kernel(int64_t M, int64_t N, int64_t K, const double* A, int64_t a_rs, int64_t a_cs,
                              const double* B, int64_t b_rs, int64_t b_cs, double* C, int64_t ldc, float* C32,
                              int64_t ldc32) {
  __shared__ double As[kT][kT + 1], Bs[kT][kT + 1];
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int64_t i = (int64_t)blockIdx.y * kT + ty, j = (int64_t)blockIdx.x * kT + tx;
  double acc = 0.0;
  for (int64_t k0 = 0; k0 < K; k0 += kT) {
    int64_t ka = k0 + tx, kb = k0 + ty;
    As[ty][tx] = (i < M && ka < K) ? A[i * a_rs + ka * a_cs] : 0.0;
    Bs[ty][tx] = (kb < K && j < N) ? B[kb * b_rs + j * b_cs] : 0.0;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kT; ++q) acc += As[ty][q] * Bs[q][tx];
    __syncthreads();
  }
  if (i < M && j < N) {
    if (C) C[i * ldc + j] = acc;
    if (C32) C32[i * ldc32 + j] = (float)acc;
  }
}

// Right-looking Cholesky in LDS followed by an in-place column-by-column inverse of R.
// flag: 0 on success, 1 if a pivot is not positive (relative to the largest diagonal).
__global__ __launch_bounds__(1024) void chol_inv64_kernel(const double* G, int l, double* Rinv, int* flag) {
  extern __shared__ double S[];  // l*l
  __shared__ double s_piv;
  __shared__ int s_bad;
  __shared__ double s_dmax;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < l * l; e += nt) S[e] = G[e];
  if (tid == 0) {
    s_bad = 0;
    double m = 0.0;
    for (int j = 0; j < l; ++j) m = fmax(m, fabs(G[j * l + j]));
    s_dmax = m;
  }
  __syncthreads();
  for (int j = 0; j < l; ++j) {
    if (tid == 0) {
      double p = S[j * l + j];
      if (!(p > 1e-30 * s_dmax) || !isfinite(p)) {
        s_bad = 1;
        p = 1.0;
      }
      s_piv = sqrt(p);
      S[j * l + j] = s_piv;
    }
    __syncthreads();
    double piv = s_piv;
    for (int c = j + 1 + tid; c < l; c += nt) S[j * l + c] /= piv;
    __syncthreads();
    // trailing update of the upper triangle: S[a][c] -= R[j][a] R[j][c], j < a <= c
    int m = l - j - 1;
    for (int e = tid; e < m * m; e += nt) {
      int a = j + 1 + e / m, c = j + 1 + e % m;
      if (c >= a) S[a * l + c] -= S[j * l + a] * S[j * l + c];
    }
    __syncthreads();
  }
  // zero the strict lower triangle
  for (int e = tid; e < l * l; e += nt) {
    int a = e / l, c = e % l;
    if (c < a) S[e] = 0.0;
  }
  __syncthreads();
  // In-place inverse of upper-triangular R, column by column:
  //   X[j][j] = 1/R[j][j];  X[i][j] = -(sum_{q=i}^{j-1} X[i][q] R[q][j]) / R[j][j]  (i < j)
  // Column j of R is read before it is overwritten; columns < j already hold X.
  __shared__ double col[256];
  for (int j = 0; j < l; ++j) {
    double rjj = S[j * l + j];
    for (int i = tid; i < j; i += nt) {
      double acc = 0.0;
      for (int q = i; q < j; ++q) acc += S[i * l + q] * S[q * l + j];
      col[i] = -acc / rjj;
    }
    __syncthreads();
    for (int i = tid; i < j; i += nt) S[i * l + j] = col[i];
    if (tid == 0) S[j * l + j] = 1.0 / rjj;
    __syncthreads();
  }
  for (int e = tid; e < l * l; e += nt) Rinv[e] = S[e];
  if (tid == 0) *flag = s_bad;
}

// Round-robin pairing: P players (P even), round t, slot s in [0, P/2): (pos s, pos P-1-s),
// player at position 0 is 0, at position q >= 1 it is 1 + (q - 1 + t) mod (P - 1).
__device__ __forceinline__ int rr_player(int pos, int t, int P) { return pos == 0 ? 0 : 1 + (pos - 1 + t) % (P - 1); }

template <bool IN_LDS>
__global__ __launch_bounds__(1024) void jacobi64_kernel(const double* B, int l, double* Aglob, double* V,
                                                        double* theta, int* order, int max_sweeps) {
  extern __shared__ double S[];
  double* A = IN_LDS ? S : Aglob;
  __shared__ double cs_c[128], cs_s[128];
  __shared__ int cs_p[128], cs_q[128];
  __shared__ double s_off, s_tot;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < l * l; e += nt) {
    A[e] = B[e];
    V[e] = (e / l == e % l) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int P = (l + 1) & ~1;
  const int half = P / 2;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    // convergence test on the off-diagonal mass
    if (tid == 0) {
      s_off = 0.0;
      s_tot = 0.0;
    }
    __syncthreads();
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < l * l; e += nt) {
      double a = A[e];
      tot += a * a;
      if (e / l != e % l) off += a * a;
    }
    off = warp_sum_d(off);
    tot = warp_sum_d(tot);
    if ((tid & 63) == 0) {
      atomicAdd(&s_off, off);
      atomicAdd(&s_tot, tot);
    }
    __syncthreads();
    if (!(s_off > 1e-30 * s_tot)) break;
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
          if (fabs(apq) > 1e-300 && fabs(apq) > 1e-18 * sqrt(fabs(app * aqq))) {
            double tau = (aqq - app) / (2.0 * apq);
            double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tt * tt);
            sn = tt * c;
          }
        }
        cs_p[s] = p;
        cs_q[s] = q;
        cs_c[s] = c;
        cs_s[s] = sn;
      }
      __syncthreads();
      // rows: row_p' = c row_p - s row_q ; row_q' = s row_p + c row_q
      for (int e = tid; e < half * l; e += nt) {
        int s = e / l, j = e % l;
        int p = cs_p[s], q = cs_q[s];
        if (q >= l || cs_s[s] == 0.0) continue;
        double c = cs_c[s], sn = cs_s[s];
        double ap = A[p * l + j], aq = A[q * l + j];
        A[p * l + j] = c * ap - sn * aq;
        A[q * l + j] = sn * ap + c * aq;
      }
      __syncthreads();
      // columns of A and of V
      for (int e = tid; e < half * l; e += nt) {
        int s = e / l, i = e % l;
        int p = cs_p[s], q = cs_q[s];
        if (q >= l || cs_s[s] == 0.0) continue;
        double c = cs_c[s], sn = cs_s[s];
        double ap = A[i * l + p], aq = A[i * l + q];
        A[i * l + p] = c * ap - sn * aq;
        A[i * l + q] = sn * ap + c * aq;
        double vp = V[i * l + p], vq = V[i * l + q];
        V[i * l + p] = c * vp - sn * vq;
        V[i * l + q] = sn * vp + c * vq;
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < l; i += nt) theta[i] = A[i * l + i];
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
  gemm64_kernel<<<grid, dim3(kT, kT), 0, st>>>(M, N, K, A, a_rs, a_cs, B, b_rs, b_cs, C, ldc, C32, ldc32);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_chol_inv64(hipStream_t st, const double* G, int l, double* Rinv, int* flag) {
  size_t bytes = (size_t)l * l * sizeof(double);
  if (l > 256 || (int64_t)bytes + 4096 > max_lds_bytes()) {
    set_error("CholeskyQR: the sketch width k + p is too large for one workgroup's LDS");
    return SCS_EINVAL;
  }
  if (bytes > 65536) SCS_HIP(hipFuncSetAttribute((const void*)chol_inv64_kernel,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  chol_inv64_kernel<<<1, 1024, bytes, st>>>(G, l, Rinv, flag);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_jacobi64(hipStream_t st, const double* B, int l, double* Awork, double* V, double* theta, int* order) {
  if (l > 256) {
    set_error("Jacobi: the sketch width k + p is too large");
    return SCS_EINVAL;
  }
  size_t bytes = (size_t)l * l * sizeof(double);
  const int sweeps = 40;
  if ((int64_t)bytes + 8192 <= max_lds_bytes()) {
    if (bytes > 65536) SCS_HIP(hipFuncSetAttribute((const void*)jacobi64_kernel<true>,
                                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    jacobi64_kernel<true><<<1, 1024, bytes, st>>>(B, l, Awork, V, theta, order, sweeps);
  } else {
    jacobi64_kernel<false><<<1, 1024, 0, st>>>(B, l, Awork, V, theta, order, sweeps);
  }
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

}  // namespace scs
