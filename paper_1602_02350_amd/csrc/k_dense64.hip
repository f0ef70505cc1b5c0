// FP64 dense algebra on the small matrices of the sketch (l = k + p <= 136):
//  * gemm64: C = A B with arbitrary strides (covers transposes), 16x16 LDS tiles;
//  * chol_inv64: G = R^T R (upper R) and R^{-1}, one workgroup, packed triangles, for CholeskyQR2
//    (Q = Y R^{-1}, twice; Fukaya, Nakatsukasa, Yanagisawa, Yamamoto 2014);
#include "scs_internal.h"

namespace scs {

namespace {

constexpr int kT = 16;

// 16x16 output tile per workgroup; the K range is split over kKZ thread slices (threadIdx.z) that
// walk interleaved 16-wide K tiles in lockstep, and their partial tiles are added in slice order.
constexpr int kKZ = 4;

__device__ __forceinline__ void gemm64_body(int bx, int by, int64_t M, int64_t N, int64_t K, const double* A,
                                            int64_t a_rs, int64_t a_cs, const double* B, int64_t b_rs,
                                            int64_t b_cs, double* C, int64_t ldc, float* C32, int64_t ldc32) {
  __shared__ double As[kKZ][kT][kT + 1], Bs[kKZ][kT][kT + 1];
  const int tx = threadIdx.x, ty = threadIdx.y, tz = threadIdx.z;
  const int64_t i = (int64_t)by * kT + ty, j = (int64_t)bx * kT + tx;
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

__global__ __launch_bounds__(kT * kT * kKZ) void gemm64_kernel(int64_t M, int64_t N, int64_t K, const double* A,
                                                               int64_t a_rs, int64_t a_cs, const double* B,
                                                               int64_t b_rs, int64_t b_cs, double* C, int64_t ldc,
                                                               float* C32, int64_t ldc32) {
  gemm64_body((int)blockIdx.x, (int)blockIdx.y, M, N, K, A, a_rs, a_cs, B, b_rs, b_cs, C, ldc, C32, ldc32);
}

// Cholesky G = R^T R (upper R), then R^{-1}, in two launches.
// chol64: one workgroup; G arrives as nparts matrices (upper triangles) that it adds in order (one:
// G itself); R packed in LDS (l (l + 1) / 2 doubles, then the l reciprocal diagonal entries),
// copied out in that layout. Right-looking with one barrier per column: phase j reads the finished
// diagonal entry p_j and the unscaled row j, updates the trailing triangle with
// S[a][c] -= (S[j][a] / p_j) S[j][c] (lanes over columns c, each holding its S[j][c] in registers,
// waves over rows a), and scales row j - 1 (which nothing reads in that phase) by 1/sqrt(p_{j-1}).
// rinv64: X = R^{-1} one column per wave, over as many workgroups as the columns need, by back
// substitution in axpy form: x = e_j, and for q = j, ..., 0: x_q *= 1/R[q][q], x_i -= R[i][q] x_q
// (i < q); lane t keeps x_t, x_{t+64}, x_{t+128} in registers and the entries of R for step q - 1 are
// read from LDS while step q runs.
// flag: 0 on success, 1 if a pivot is not positive relative to the largest diagonal entry of G
// (that pivot is replaced by 1 so the factor stays finite).
constexpr int kCholThreads = 1024;
constexpr int kRinvWaves = 4;  // columns of R^{-1} per workgroup

__device__ __forceinline__ int packed_up(int i, int j, int l) { return i * (2 * l - i + 1) / 2 + (j - i); }
// offset of row i of the packed triangle, so that R[i][j] = S[packed_row(i, l) + j] for j >= i
__device__ __forceinline__ int packed_row(int i, int l) { return i * (2 * l - i - 1) / 2; }

__device__ __forceinline__ double readlane_d(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ void chol64_body(double* S /* LDS */, const double* part, int nparts, int l, double* Rp,
                                            int* flag) {
  __shared__ double s_dmax;
  double* rdiag = S + l * (l + 1) / 2;
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, nwave = nt >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  for (int e = tid; e < l * l; e += nt) {
    int i = e / l, j = e % l;
    if (j >= i) {
      double g = 0.0;
#pragma unroll 8
      for (int q = 0; q < nparts; ++q) g += part[(int64_t)q * l * l + e];
      S[packed_row(i, l) + j] = g;
    }
  }
  __syncthreads();
  if (wave == 0) {  // largest diagonal entry: one wave, lanes over the diagonal
    double m = 0.0;
    for (int j = lane; j < l; j += 64) m = fmax(m, fabs(S[packed_row(j, l) + j]));
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    if (lane == 0) s_dmax = m;
  }
  __syncthreads();
  const double dmax = s_dmax;
  int bad = 0;
  auto pivot = [&](int j) {
    double p = S[packed_row(j, l) + j];
    if (!(p > 1e-30 * dmax) || !isfinite(p)) {
      bad = 1;
      p = 1.0;
    }
    return p;
  };
  // row r scaled by 1 / sqrt(p_r), its diagonal set to sqrt(p_r) (both formed when p_r is read)
  auto finish_row = [&](int r, double sp, double isp) {
    const int row = packed_row(r, l);
    for (int c = r + tid; c < l; c += nt) S[row + c] = c == r ? sp : S[row + c] * isp;
    if (tid == 0) rdiag[r] = isp;
  };
  double sp_prev = 1.0, isp_prev = 1.0;
  for (int j = 0; j < l; ++j) {
    const double p = pivot(j), ip = 1.0 / p;
    const double sp = sqrt(p), isp = 1.0 / sp;  // independent of the update: overlaps it
    const int rowj = packed_row(j, l);
    constexpr int kCC = 3;  // column chunks of 64: l <= 192
    double sj[kCC];
#pragma unroll
    for (int q = 0; q < kCC; ++q) {
      const int c = j + 1 + lane + 64 * q;
      sj[q] = c < l ? S[rowj + c] : 0.0;
    }
#pragma unroll 4
    for (int a = j + 1 + wave; a < l; a += nwave) {
      const double ra = S[rowj + a] * ip;
      const int rowa = packed_row(a, l);
#pragma unroll
      for (int q = 0; q < kCC; ++q) {
        const int c = j + 1 + lane + 64 * q;
        if (c < l && c >= a) S[rowa + c] -= ra * sj[q];
      }
    }
    if (j > 0) finish_row(j - 1, sp_prev, isp_prev);
    sp_prev = sp;
    isp_prev = isp;
    __syncthreads();
  }
  finish_row(l - 1, sp_prev, isp_prev);
  __syncthreads();
  for (int e = tid; e < l * (l + 1) / 2 + l; e += nt) Rp[e] = S[e];
  if (tid == 0) *flag = bad;
}

// gate (nullable): the factor is formed only while *gate != 0
__global__ __launch_bounds__(kCholThreads) void chol64_kernel(const double* part, int nparts, int l, double* Rp,
                                                              int* flag, const int* gate) {
  if (gate && *gate == 0) return;
  extern __shared__ double dyn[];
  chol64_body(dyn, part, nparts, l, Rp, flag);
}

// Second pass of CholeskyQR2 when the first has already left Q1 orthonormal to working accuracy:
// G = Q1^T Q1 = I + E (upper triangle of G read, E symmetric), and l max |E_ij| bounds ||E||_2.
// (I + E)^{-1/2} = I - E/2 + 3 E^2/8 - ... (binomial series): up to kLowdinTol1 the first-order M = I - E/2
// is within 3/8 ||E||^2 <= 4e-15 of it, up to kLowdinTol2 the second-order M within 5/16 ||E||^3 <= 4e-16.
// Q = Q1 M is then orthonormal to FP64 rounding with the span of Q1 (symmetric orthogonalization); M goes
// to Minv, the pass's breakdown flag to 0 and *use_chol to 0. Otherwise (and for non-finite E)
// *use_chol = 1, and the Cholesky factor and its inverse, gated on that flag, write R^{-1} to Minv
// instead. One workgroup; E in LDS (l^2 doubles). The E^2 term costs 6 us at l = 55 and about 100 us
// at l = 133 (its broadcast LDS reads each move a full wave of data), still under the Cholesky's 280.
constexpr double kLowdinTol1 = 1e-7;
constexpr double kLowdinTol2 = 1e-5;

__device__ __forceinline__ void lowdin64_body(double* E /* LDS, l x l */, const double* G, int l, double* Minv,
                                              int* flag, int* use_chol) {
  __shared__ double sred[kCholThreads / 64];
  __shared__ int s_small;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nt = blockDim.x;
  double m = 0.0;
  bool bad = false;
  // upper triangle of G read row-major (coalesced), mirrored into the lower triangle of E in LDS
  for (int e = tid; e < l * l; e += nt) {
    const int i = e / l, j = e - i * l;
    if (i <= j) {
      const double v = G[e] - (i == j ? 1.0 : 0.0);
      E[e] = v;
      E[j * l + i] = v;
      if (!isfinite(v)) bad = true;
      m = fmax(m, fabs(v));
    }
  }
  if (bad) m = INFINITY;
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
  if (lane == 0) sred[wave] = m;
  __syncthreads();
  if (tid == 0) {
    double mx = 0.0;
    for (int w = 0; w < nt / 64; ++w) mx = fmax(mx, sred[w]);
    const double r = (double)l * mx;
    const int order = r <= kLowdinTol1 ? 1 : (r <= kLowdinTol2 ? 2 : 0);  // series terms kept (0: Cholesky)
    s_small = order;
    *use_chol = order ? 0 : 1;
    if (order) *flag = 0;
  }
  __syncthreads();
  const int order = s_small;
  if (order == 0) return;
  if (order == 1) {
    for (int e = tid; e < l * l; e += nt) {
      const int i = e / l, j = e - i * l;
      Minv[e] = (i == j ? 1.0 : 0.0) - 0.5 * E[e];
    }
    return;
  }
  // E^2 by waves over tasks of 8 rows x 64 columns: lane j reads E[t][j] (contiguous across the wave)
  // and the 8 row entries E[i][t] are wave-uniform; each entry sums over t in order
  constexpr int kRB = 8;
  const int nrb = (l + kRB - 1) / kRB, ncb = (l + 63) / 64, nwave = nt >> 6;
  for (int task = wave; task < nrb * ncb; task += nwave) {
    const int rb = task / ncb, cb = task - rb * ncb;
    const int j = cb * 64 + lane, jc = j < l ? j : l - 1;
    double acc[kRB];
#pragma unroll
    for (int q = 0; q < kRB; ++q) acc[q] = 0.0;
    for (int t = 0; t < l; ++t) {
      const double b = E[t * l + jc];
#pragma unroll
      for (int q = 0; q < kRB; ++q) {
        const int i = rb * kRB + q, ic = i < l ? i : l - 1;
        acc[q] += E[ic * l + t] * b;
      }
    }
    if (j < l) {
#pragma unroll
      for (int q = 0; q < kRB; ++q) {
        const int i = rb * kRB + q;
        if (i < l) Minv[i * l + j] = (i == j ? 1.0 : 0.0) - 0.5 * E[i * l + j] + 0.375 * acc[q];
      }
    }
  }
}

__global__ __launch_bounds__(kCholThreads) void lowdin64_kernel(const double* G, int l, double* Minv, int* flag,
                                                                int* use_chol) {
  extern __shared__ double dyn[];
  lowdin64_body(dyn, G, l, Minv, flag, use_chol);
}

__device__ __forceinline__ void rinv64_body(double* S /* LDS */, int bx, const double* Rp, int l, double* Rinv) {
  double* rdiag = S + l * (l + 1) / 2;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  for (int e = tid; e < l * (l + 1) / 2 + l; e += blockDim.x) S[e] = Rp[e];
  __syncthreads();
  const int j = bx * kRinvWaves + wave;
  if (j >= l) return;
  int roff[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) roff[r] = packed_row(min(lane + 64 * r, l - 1), l);
  // S reads use in-bounds clamped addresses (lanes past the triangle read a valid entry that the
  // update then ignores), so the loop has no per-lane branches
  double x[3], sv[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const int i = lane + 64 * r;
    x[r] = i == j ? 1.0 : 0.0;
    sv[r] = S[roff[r] + max(j, min(i, l - 1))];
  }
  double rq = rdiag[j];
  for (int q = j; q >= 0; --q) {
    // entries for step q - 1, read while step q runs
    double sn[3];
    const int qn = max(q - 1, 0);
#pragma unroll
    for (int r = 0; r < 3; ++r) sn[r] = S[roff[r] + max(qn, min(lane + 64 * r, l - 1))];
    const double rq_next = rdiag[qn];
    const int slot = q >> 6, owner = q & 63;  // uniform across the wave
    const double mine = slot == 0 ? x[0] : (slot == 1 ? x[1] : x[2]);
    const double xq = readlane_d(mine, owner) * rq;
    if (lane == owner) {
      if (slot == 0) x[0] = xq;
      else if (slot == 1) x[1] = xq;
      else x[2] = xq;
    }
#pragma unroll
    for (int r = 0; r < 3; ++r)
      if (lane + 64 * r < q) x[r] -= sv[r] * xq;
#pragma unroll
    for (int r = 0; r < 3; ++r) sv[r] = sn[r];
    rq = rq_next;
  }
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const int i = lane + 64 * r;
    if (i < l) Rinv[(int64_t)i * l + j] = i <= j ? x[r] : 0.0;
  }
}

__global__ __launch_bounds__(64 * kRinvWaves) void rinv64_kernel(const double* Rp, int l, double* Rinv,
                                                                const int* gate) {
  if (gate && *gate == 0) return;
  extern __shared__ double dyn[];
  rinv64_body(dyn, (int)blockIdx.x, Rp, l, Rinv);
}

// Partial Gram matrices of Y d x l (row-major, ld l): each workgroup stages kGramRows rows of Y in LDS
// and forms their Y_r^T Y_r (upper triangle, one thread per entry, rows in order); gram_sum64 adds
// them in workgroup order, one thread per entry (loads of eight partials in flight), and mirrors.
constexpr int kGramRows = 32;
__host__ __device__ __forceinline__ int64_t gram64_parts_dev(int64_t d) { return (d + kGramRows - 1) / kGramRows; }

__device__ __forceinline__ void gram_part64_body(double* Ys /* LDS */, int bx, const double* Y, int64_t d, int l,
                                                 double* part) {
  const int64_t r0 = (int64_t)bx * kGramRows;
  const int nr = (int)(d - r0 < kGramRows ? d - r0 : kGramRows);
  for (int e = threadIdx.x; e < nr * l; e += blockDim.x) Ys[e] = Y[r0 * l + e];
  __syncthreads();
  double* out = part + (int64_t)bx * l * l;
  for (int e = threadIdx.x; e < l * l; e += blockDim.x) {
    const int i = e / l, j = e % l;
    if (j < i) continue;
    double acc = 0.0;
    for (int r = 0; r < nr; ++r) acc += Ys[r * l + i] * Ys[r * l + j];
    out[e] = acc;
  }
}

__global__ __launch_bounds__(256) void gram_part64_kernel(const double* Y, int64_t d, int l, double* part) {
  extern __shared__ double dyn[];
  gram_part64_body(dyn, (int)blockIdx.x, Y, d, l, part);
}

__device__ __forceinline__ void gram_sum64_body(int e, const double* part, int nparts, int l, double* G) {
  if (e >= l * l) return;
  const int i = e / l, j = e % l;
  if (j < i) return;
  double g = 0.0;
#pragma unroll 8
  for (int p = 0; p < nparts; ++p) g += part[(int64_t)p * l * l + e];
  G[(int64_t)i * l + j] = g;
  G[(int64_t)j * l + i] = g;
}

__global__ __launch_bounds__(256) void gram_sum64_kernel(const double* part, int nparts, int l, double* G) {
  gram_sum64_body((int)(blockIdx.x * blockDim.x + threadIdx.x), part, nparts, l, G);
}

// CholeskyQR2 of many problems at once (jobs[blockIdx.y or .z]); the per-problem arithmetic is the
// one-problem kernels'. Workgroups past a problem's own grid return.
__global__ __launch_bounds__(256) void gram_part64_batched_kernel(const CholJob* jobs, int pass) {
  extern __shared__ double dyn[];
  const CholJob jb = jobs[blockIdx.y];
  if ((int64_t)blockIdx.x >= gram64_parts_dev(jb.d)) return;
  gram_part64_body(dyn, (int)blockIdx.x, pass == 0 ? jb.Y : jb.Q1, jb.d, jb.l, jb.Gp);
}

__global__ __launch_bounds__(256) void gram_sum64_batched_kernel(const CholJob* jobs) {
  const CholJob jb = jobs[blockIdx.y];
  gram_sum64_body((int)(blockIdx.x * blockDim.x + threadIdx.x), jb.Gp, (int)gram64_parts_dev(jb.d), jb.l, jb.G);
}

// pass 1 runs only where the job's gate asks for the Cholesky (lowdin64_batched_kernel decides)
__global__ __launch_bounds__(kCholThreads) void chol64_batched_kernel(const CholJob* jobs, int pass) {
  extern __shared__ double dyn[];
  const CholJob jb = jobs[blockIdx.x];
  if (pass == 1 && *jb.gate == 0) return;
  chol64_body(dyn, jb.G, 1, jb.l, jb.Rp, jb.flags + pass);
}

__global__ __launch_bounds__(kCholThreads) void lowdin64_batched_kernel(const CholJob* jobs) {
  extern __shared__ double dyn[];
  const CholJob jb = jobs[blockIdx.x];
  lowdin64_body(dyn, jb.G, jb.l, jb.Rinv, jb.flags + 1, jb.gate);
}

__global__ __launch_bounds__(64 * kRinvWaves) void rinv64_batched_kernel(const CholJob* jobs, int pass) {
  extern __shared__ double dyn[];
  const CholJob jb = jobs[blockIdx.y];
  if ((int)blockIdx.x * kRinvWaves >= jb.l) return;  // uniform: before any barrier
  if (pass == 1 && *jb.gate == 0) return;
  rinv64_body(dyn, (int)blockIdx.x, jb.Rp, jb.l, jb.Rinv);
}

// step 0: Q1 = Y R1^{-1}; 1: Q = Q1 R2^{-1}; 2: Q^T in FP32 as R2^{-T} Q1^T
__global__ __launch_bounds__(kT * kT * kKZ) void gemm64_chol_batched_kernel(const CholJob* jobs, int step) {
  const CholJob jb = jobs[blockIdx.z];
  const int64_t d = jb.d;
  const int l = jb.l;
  if (step == 0) {
    if ((int64_t)blockIdx.y * kT >= d || (int)blockIdx.x * kT >= l) return;
    gemm64_body((int)blockIdx.x, (int)blockIdx.y, d, l, l, jb.Y, l, 1, jb.Rinv, l, 1, jb.Q1, l, nullptr, 0);
  } else if (step == 1) {
    if ((int64_t)blockIdx.y * kT >= d || (int)blockIdx.x * kT >= l) return;
    gemm64_body((int)blockIdx.x, (int)blockIdx.y, d, l, l, jb.Q1, l, 1, jb.Rinv, l, 1, jb.Q, jb.ldq, nullptr, 0);
  } else {
    if (!jb.QT || (int)blockIdx.y * kT >= l || (int64_t)blockIdx.x * kT >= d) return;
    gemm64_body((int)blockIdx.x, (int)blockIdx.y, l, d, l, jb.Rinv, 1, l, jb.Q1, 1, l, nullptr, 0, jb.QT, d);
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

// y += alpha x (FP64, count entries)
__global__ void axpy64_kernel(int64_t count, double alpha, const double* x, double* y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) y[i] += alpha * x[i];
}

// dst (rows x cols, leading dimension ldd) = src (rows x cols, leading dimension lds), FP64
__global__ void copy64_kernel(int64_t rows, int64_t cols, const double* src, int64_t lds, double* dst, int64_t ldd) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t r = e / cols, c = e % cols;
  dst[r * ldd + c] = src[r * lds + c];
}

// dst (cols x rows, FP32, row-major) = src^T, src rows x cols FP64 with leading dimension lds
__global__ void transpose64to32_kernel(int64_t rows, int64_t cols, const double* src, int64_t lds, float* dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t c = e / rows, r = e % rows;   // consecutive threads write consecutive dst entries
  dst[c * rows + r] = (float)src[r * lds + c];
}

// dst[0] = 1 if any of src[0 .. count) is set, dst[1] = 0
__global__ void or_flags_kernel(const int* src, int count, int* dst) {
  if (threadIdx.x != 0) return;
  int any = 0;
  for (int i = 0; i < count; ++i) any |= src[i] != 0;
  dst[0] = any;
  dst[1] = 0;
}

}  // namespace

int launch_axpy64(hipStream_t st, int64_t count, double alpha, const double* x, double* y) {
  if (count <= 0) return SCS_OK;
  axpy64_kernel<<<(unsigned)cdiv(count, 256), 256, 0, st>>>(count, alpha, x, y);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_copy64(hipStream_t st, int64_t rows, int64_t cols, const double* src, int64_t lds, double* dst,
                  int64_t ldd) {
  if (rows * cols <= 0) return SCS_OK;
  copy64_kernel<<<(unsigned)cdiv(rows * cols, 256), 256, 0, st>>>(rows, cols, src, lds, dst, ldd);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_transpose64to32(hipStream_t st, int64_t rows, int64_t cols, const double* src, int64_t lds, float* dst) {
  if (rows * cols <= 0) return SCS_OK;
  transpose64to32_kernel<<<(unsigned)cdiv(rows * cols, 256), 256, 0, st>>>(rows, cols, src, lds, dst);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_or_flags(hipStream_t st, const int* src, int count, int* dst) {
  or_flags_kernel<<<1, 64, 0, st>>>(src, count, dst);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_gemm64(hipStream_t st, int64_t M, int64_t N, int64_t K, const double* A, int64_t a_rs, int64_t a_cs,
                  const double* B, int64_t b_rs, int64_t b_cs, double* C, int64_t ldc, float* C32,
                  int64_t ldc32) {
  if (M <= 0 || N <= 0) return SCS_OK;
  dim3 grid((unsigned)cdiv(N, kT), (unsigned)cdiv(M, kT));
  gemm64_kernel<<<grid, dim3(kT, kT, kKZ), 0, st>>>(M, N, K, A, a_rs, a_cs, B, b_rs, b_cs, C, ldc, C32, ldc32);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int64_t gram64_parts(int64_t d) { return gram64_parts_dev(d); }

int launch_gram64(hipStream_t st, const double* Y, int64_t d, int l, double* part, double* G) {
  if (l <= 0 || d <= 0) return SCS_OK;
  const size_t bytes = (size_t)kGramRows * l * sizeof(double);
  if (bytes > 65536)
    SCS_HIP(hipFuncSetAttribute((const void*)gram_part64_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)bytes));
  gram_part64_kernel<<<(unsigned)gram64_parts(d), 256, bytes, st>>>(Y, d, l, part);
  SCS_HIP(hipGetLastError());
  gram_sum64_kernel<<<(unsigned)cdiv((int64_t)l * l, 256), 256, 0, st>>>(part, (int)gram64_parts(d), l, G);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_lowdin64(hipStream_t st, const double* G, int l, double* Minv, int* flag, int* use_chol) {
  const size_t bytes = (size_t)l * l * sizeof(double);
  if (l < 1 || (int64_t)bytes + 1024 > max_lds_bytes()) {
    set_error("CholeskyQR: the sketch width k + p is too large for one workgroup");
    return SCS_EINVAL;
  }
  if (bytes > 65536)
    SCS_HIP(hipFuncSetAttribute((const void*)lowdin64_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  lowdin64_kernel<<<1, kCholThreads, bytes, st>>>(G, l, Minv, flag, use_chol);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_chol_inv64(hipStream_t st, const double* part, int nparts, int l, double* Rp, double* Rinv, int* flag,
                      const int* gate) {
  const size_t bytes = ((size_t)l * (l + 1) / 2 + l) * sizeof(double);
  if (l > 192 || (int64_t)bytes + 1024 > max_lds_bytes()) {
    set_error("CholeskyQR: the sketch width k + p is too large for one workgroup");
    return SCS_EINVAL;
  }
  if (bytes > 65536) {
    SCS_HIP(hipFuncSetAttribute((const void*)chol64_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    SCS_HIP(hipFuncSetAttribute((const void*)rinv64_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  }
  chol64_kernel<<<1, kCholThreads, bytes, st>>>(part, nparts, l, Rp, flag, gate);
  SCS_HIP(hipGetLastError());
  rinv64_kernel<<<(unsigned)cdiv(l, kRinvWaves), 64 * kRinvWaves, bytes, st>>>(Rp, l, Rinv, gate);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_cholqr2_batched(hipStream_t st, const CholJob* jobs, int nj, int64_t max_d, int max_l) {
  if (nj <= 0) return SCS_OK;
  const size_t cbytes = ((size_t)max_l * (max_l + 1) / 2 + max_l) * sizeof(double);
  const size_t gbytes = (size_t)kGramRows * max_l * sizeof(double);
  if (max_l > 192 || (int64_t)cbytes + 1024 > max_lds_bytes()) {
    set_error("CholeskyQR: the sketch width k + p is too large for one workgroup");
    return SCS_EINVAL;
  }
  if (cbytes > 65536) {
    SCS_HIP(hipFuncSetAttribute((const void*)chol64_batched_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)cbytes));
    SCS_HIP(hipFuncSetAttribute((const void*)rinv64_batched_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)cbytes));
  }
  if (gbytes > 65536)
    SCS_HIP(hipFuncSetAttribute((const void*)gram_part64_batched_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)gbytes));
  const size_t lbytes = (size_t)max_l * max_l * sizeof(double);
  if ((int64_t)lbytes + 1024 > max_lds_bytes()) {
    set_error("CholeskyQR: the sketch width k + p is too large for one workgroup");
    return SCS_EINVAL;
  }
  if (lbytes > 65536)
    SCS_HIP(hipFuncSetAttribute((const void*)lowdin64_batched_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lbytes));
  for (int pass = 0; pass < 2; ++pass) {
    gram_part64_batched_kernel<<<dim3((unsigned)gram64_parts_dev(max_d), (unsigned)nj), 256, gbytes, st>>>(jobs, pass);
    SCS_HIP(hipGetLastError());
    gram_sum64_batched_kernel<<<dim3((unsigned)cdiv((int64_t)max_l * max_l, 256), (unsigned)nj), 256, 0, st>>>(jobs);
    SCS_HIP(hipGetLastError());
    if (pass == 1) {
      lowdin64_batched_kernel<<<(unsigned)nj, kCholThreads, lbytes, st>>>(jobs);
      SCS_HIP(hipGetLastError());
    }
    chol64_batched_kernel<<<(unsigned)nj, kCholThreads, cbytes, st>>>(jobs, pass);
    SCS_HIP(hipGetLastError());
    rinv64_batched_kernel<<<dim3((unsigned)cdiv(max_l, kRinvWaves), (unsigned)nj), 64 * kRinvWaves, cbytes, st>>>(
        jobs, pass);
    SCS_HIP(hipGetLastError());
    gemm64_chol_batched_kernel<<<dim3((unsigned)cdiv(max_l, kT), (unsigned)cdiv(max_d, kT), (unsigned)nj),
                                 dim3(kT, kT, kKZ), 0, st>>>(jobs, pass);
    SCS_HIP(hipGetLastError());
  }
  gemm64_chol_batched_kernel<<<dim3((unsigned)cdiv(max_d, kT), (unsigned)cdiv(max_l, kT), (unsigned)nj),
                               dim3(kT, kT, kKZ), 0, st>>>(jobs, 2);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

}  // namespace scs
