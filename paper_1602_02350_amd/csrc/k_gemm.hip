// MFMA GEMMs of the sketch and of the preconditioning step (gfx950, 64-wide waves).
//
//  gemm_nt_longk : C[M x N] = A[M x K] Bt[N x K]^T, N <= 144, K long   (X Omega, X Q, W V_k)
//  gemm_nt_wide  : C = alpha A Bt^T + beta C0 (+ diag on i == j), K <= 160, N long, optional BF16
//                  output and row norms ||C_i||^2 of the stored rows  (x~_i = x_i/s + Z D U~^T; b_j rows)
//  gemm_tn_splitk: partial[chunk] = A[rows in chunk]^T B[rows in chunk]  (X^T (X Omega), (XQ)^T (XQ))
//
// Operands are staged through LDS with coalesced float4 loads. Each lane feeds the MFMA four
// consecutive k values read as one float4 ("permuted K": MFMA r of the FP32 16x16x4 instruction
// consumes k = kq + 4*(lane/16) + r, which sums the same 16 products as the natural order); the
// BF16 16x16x16 instruction takes the same four values rounded to BF16 (RNE) with FP32 accumulation.
// Output layout of both 16x16 instructions: acc[r] = C[4*(lane/16) + r][lane % 16].
#include "scs_internal.h"

namespace scs {

namespace {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef short s4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short bf16s(float f) { return (short)f32_to_bf16(f); }

template <bool BF16>
__device__ __forceinline__ void mfma16(const float4& a, const float4& b, f4v& acc) {
  if constexpr (BF16) {
    s4v av = {bf16s(a.x), bf16s(a.y), bf16s(a.z), bf16s(a.w)};
    s4v bv = {bf16s(b.x), bf16s(b.y), bf16s(b.z), bf16s(b.w)};
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
  } else {
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b.z, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b.w, acc, 0, 0, 0);
  }
}

// Guarded load of 4 consecutive floats of row `row` starting at column `col`.
__device__ __forceinline__ float4 load4(const float* base, int64_t ld, int64_t rows, int64_t cols, int64_t row,
                                        int64_t col, bool aligned) {
  float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
  if (row >= rows) return v;
  const float* p = base + row * ld + col;
  if (aligned && col + 3 < cols) return *reinterpret_cast<const float4*>(p);
  if (col + 0 < cols) v.x = p[0];
  if (col + 1 < cols) v.y = p[1];
  if (col + 2 < cols) v.z = p[2];
  if (col + 3 < cols) v.w = p[3];
  return v;
}

// ------------------------------------------------------------------ NT, long K
constexpr int kLkBM = 128, kLkBK = 32, kLkPad = 4;

template <int NB, bool BF16>
__global__ __launch_bounds__(256) void gemm_nt_longk_kernel(const float* __restrict__ A, int64_t M, int64_t K,
                                                            int64_t lda, const float* __restrict__ Bt, int64_t N,
                                                            int64_t ldb, float* __restrict__ C, int64_t ldc,
                                                            bool a_al, bool b_al) {
  constexpr int BN = NB * 16;
  constexpr int LDS_W = kLkBK + kLkPad;
  __shared__ float As[kLkBM * LDS_W];
  __shared__ float Bs[BN * LDS_W];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t m0 = (int64_t)blockIdx.x * kLkBM;
  constexpr int A_SLOTS = kLkBM * (kLkBK / 4) / 256;           // 4
  constexpr int B_SLOTS = (BN * (kLkBK / 4) + 255) / 256;      // <= 5
  float4 ra[A_SLOTS], rb[B_SLOTS];
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < A_SLOTS; ++q) {
      int e = tid + 256 * q, r = e >> 3, c4 = e & 7;
      ra[q] = load4(A, lda, M, K, m0 + r, k0 + 4 * c4, a_al);
    }
#pragma unroll
    for (int q = 0; q < B_SLOTS; ++q) {
      int e = tid + 256 * q, r = e >> 3, c4 = e & 7;
      rb[q] = e < BN * 8 ? load4(Bt, ldb, N, K, r, k0 + 4 * c4, b_al) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int q = 0; q < A_SLOTS; ++q) {
      int e = tid + 256 * q, r = e >> 3, c4 = e & 7;
      *reinterpret_cast<float4*>(&As[r * LDS_W + 4 * c4]) = ra[q];
    }
#pragma unroll
    for (int q = 0; q < B_SLOTS; ++q) {
      int e = tid + 256 * q, r = e >> 3, c4 = e & 7;
      if (e < BN * 8) *reinterpret_cast<float4*>(&Bs[r * LDS_W + 4 * c4]) = rb[q];
    }
  };
  f4v acc[2][NB];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[i][j] = f4v{0.f, 0.f, 0.f, 0.f};

  fetch(0);
  for (int64_t k0 = 0; k0 < K; k0 += kLkBK) {
    __syncthreads();
    stash();
    __syncthreads();
    if (k0 + kLkBK < K) fetch(k0 + kLkBK);
#pragma unroll
    for (int kq = 0; kq < kLkBK; kq += 16) {
      const int ko = kq + 4 * (lane >> 4);
      float4 a0 = *reinterpret_cast<const float4*>(&As[(wave * 32 + (lane & 15)) * LDS_W + ko]);
      float4 a1 = *reinterpret_cast<const float4*>(&As[(wave * 32 + 16 + (lane & 15)) * LDS_W + ko]);
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) {
        float4 b = *reinterpret_cast<const float4*>(&Bs[(cb * 16 + (lane & 15)) * LDS_W + ko]);
        mfma16<BF16>(a0, b, acc[0][cb]);
        mfma16<BF16>(a1, b, acc[1][cb]);
      }
    }
  }
#pragma unroll
  for (int rbk = 0; rbk < 2; ++rbk)
#pragma unroll
    for (int cb = 0; cb < NB; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int64_t row = m0 + wave * 32 + rbk * 16 + 4 * (lane >> 4) + r;
        int64_t col = cb * 16 + (lane & 15);
        if (row < M && col < N) C[row * ldc + col] = acc[rbk][cb][r];
      }
}

// ------------------------------------------------------------------ NT, wide N, short K
constexpr int kWdBM = 64, kWdBN = 64;

template <bool BF16, bool OUT_BF16>
__global__ __launch_bounds__(256) void gemm_nt_wide_kernel(const float* __restrict__ A, int64_t M, int64_t K,
                                                           int64_t lda, const float* __restrict__ Bt, int64_t N,
                                                           int64_t ldb, float alpha, const float* __restrict__ C0,
                                                           int64_t ldc0, float beta, const double* beta_dev,
                                                           float diag, const double* diag_dev, void* Cout,
                                                           int64_t ldc, float* __restrict__ rownorm2, int KP,
                                                           bool a_al, bool b_al, bool c0_al, bool out_al) {
  extern __shared__ float S[];
  const int LW = KP + 4;
  constexpr int CW = kWdBN + 4;
  float* As = S;                  // kWdBM x LW
  float* Bs = S + kWdBM * LW;     // kWdBN x LW
  float* Cs = Bs + kWdBN * LW;    // kWdBM x CW: the MFMA tile, re-read by rows for the epilogue
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t m0 = (int64_t)blockIdx.x * kWdBM;
  if (beta_dev) beta = (float)beta_dev[0];
  if (diag_dev) diag = (float)diag_dev[0];
  const int kv = KP / 4;
  for (int e = tid; e < kWdBM * kv; e += 256) {
    int r = e / kv, c4 = e % kv;
    *reinterpret_cast<float4*>(&As[r * LW + 4 * c4]) = load4(A, lda, M, K, m0 + r, 4 * c4, a_al);
  }
  // epilogue mapping: lane owns columns cc..cc+3 of rows 4p + lane/16 (p = 0..3) of its wave's 16 rows,
  // so 16 lanes move one contiguous 256-byte row segment
  const int cc = 4 * (lane & 15);
  float rn[4] = {0.f, 0.f, 0.f, 0.f};
  for (int64_t n0 = 0; n0 < N; n0 += kWdBN) {
    __syncthreads();
    for (int e = tid; e < kWdBN * kv; e += 256) {
      int r = e / kv, c4 = e % kv;
      *reinterpret_cast<float4*>(&Bs[r * LW + 4 * c4]) = load4(Bt, ldb, N, K, n0 + r, 4 * c4, b_al);
    }
    __syncthreads();
    f4v acc[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) acc[cb] = f4v{0.f, 0.f, 0.f, 0.f};
    for (int kq = 0; kq < KP; kq += 16) {
      const int ko = kq + 4 * (lane >> 4);
      float4 a = *reinterpret_cast<const float4*>(&As[(wave * 16 + (lane & 15)) * LW + ko]);
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        float4 b = *reinterpret_cast<const float4*>(&Bs[(cb * 16 + (lane & 15)) * LW + ko]);
        mfma16<BF16>(a, b, acc[cb]);
      }
    }
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) Cs[(wave * 16 + 4 * (lane >> 4) + r) * CW + cb * 16 + (lane & 15)] = acc[cb][r];
    __syncthreads();
    const int64_t col = n0 + cc;
    if (col < N) {
      const bool full = col + 3 < N;
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const int rl = wave * 16 + 4 * p + (lane >> 4);
        const int64_t row = m0 + rl;
        if (row >= M) continue;
        float4 t = *reinterpret_cast<const float4*>(&Cs[rl * CW + cc]);
        float v[4] = {alpha * t.x, alpha * t.y, alpha * t.z, alpha * t.w};
        if (C0) {
          float4 c = load4(C0, ldc0, M, N, row, col, c0_al);
          v[0] = fmaf(beta, c.x, v[0]);
          v[1] = fmaf(beta, c.y, v[1]);
          v[2] = fmaf(beta, c.z, v[2]);
          v[3] = fmaf(beta, c.w, v[3]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (row == col + q) v[q] += diag;
        if constexpr (OUT_BF16) {
          uint16_t h[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            h[q] = f32_to_bf16(v[q]);
            v[q] = bf16_to_f32(h[q]);
          }
          uint16_t* o = reinterpret_cast<uint16_t*>(Cout) + row * ldc + col;
          if (full && out_al) {
            uint2 w;
            w.x = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
            w.y = (uint32_t)h[2] | ((uint32_t)h[3] << 16);
            *reinterpret_cast<uint2*>(o) = w;
          } else {
#pragma unroll
            for (int q = 0; q < 4; ++q)
              if (col + q < N) o[q] = h[q];
          }
        } else {
          float* o = reinterpret_cast<float*>(Cout) + row * ldc + col;
          if (full && out_al) {
            *reinterpret_cast<float4*>(o) = make_float4(v[0], v[1], v[2], v[3]);
          } else {
#pragma unroll
            for (int q = 0; q < 4; ++q)
              if (col + q < N) o[q] = v[q];
          }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (col + q < N) rn[p] = fmaf(v[q], v[q], rn[p]);
      }
    }
  }
  if (rownorm2) {
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      float t = rn[p];
      t += __shfl_xor(t, 1);
      t += __shfl_xor(t, 2);
      t += __shfl_xor(t, 4);
      t += __shfl_xor(t, 8);
      int64_t row = m0 + wave * 16 + 4 * p + (lane >> 4);
      if ((lane & 15) == 0 && row < M) rownorm2[row] = t;
    }
  }
}

// ------------------------------------------------------------------ TN split-K
constexpr int kTnBM = 64, kTnBK = 16;

template <int NB, bool BF16>
__global__ __launch_bounds__(256) void gemm_tn_splitk_kernel(const float* __restrict__ A, int64_t R, int64_t M,
                                                             int64_t lda, const float* __restrict__ B, int64_t N,
                                                             int64_t ldb, float* __restrict__ partial,
                                                             int64_t chunk_rows, bool a_al, bool b_al) {
  constexpr int BN = NB * 16;
  constexpr int AW = kTnBM + 4, BW = BN + 4;
  __shared__ float As[kTnBK * AW];
  __shared__ float Bs[kTnBK * BW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t m0 = (int64_t)blockIdx.x * kTnBM;
  const int64_t r0 = (int64_t)blockIdx.y * chunk_rows;
  const int64_t r1 = r0 + chunk_rows < R ? r0 + chunk_rows : R;
  constexpr int B_SLOTS = (kTnBK * BN / 4 + 255) / 256;
  f4v acc[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) acc[j] = f4v{0.f, 0.f, 0.f, 0.f};
  float4 ra, rb[B_SLOTS];
  auto fetch = [&](int64_t k0) {
    {
      int r = tid >> 4, c4 = tid & 15;  // 16 rows x 16 float4
      int64_t row = k0 + r;
      ra = row < r1 ? load4(A, lda, R, M, row, m0 + 4 * c4, a_al) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int q = 0; q < B_SLOTS; ++q) {
      int e = tid + 256 * q;
      int r = e / (BN / 4), c4 = e % (BN / 4);
      int64_t row = k0 + r;
      rb[q] = (e < kTnBK * BN / 4 && row < r1) ? load4(B, ldb, R, N, row, 4 * c4, b_al)
                                               : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  auto stash = [&]() {
    {
      int r = tid >> 4, c4 = tid & 15;
      *reinterpret_cast<float4*>(&As[r * AW + 4 * c4]) = ra;
    }
#pragma unroll
    for (int q = 0; q < B_SLOTS; ++q) {
      int e = tid + 256 * q;
      int r = e / (BN / 4), c4 = e % (BN / 4);
      if (e < kTnBK * BN / 4) *reinterpret_cast<float4*>(&Bs[r * BW + 4 * c4]) = rb[q];
    }
  };
  if (r0 < r1) fetch(r0);
  for (int64_t k0 = r0; k0 < r1; k0 += kTnBK) {
    __syncthreads();
    stash();
    __syncthreads();
    if (k0 + kTnBK < r1) fetch(k0 + kTnBK);
    const int g = lane >> 4, mi = wave * 16 + (lane & 15);
    float4 a = make_float4(As[(4 * g + 0) * AW + mi], As[(4 * g + 1) * AW + mi], As[(4 * g + 2) * AW + mi],
                           As[(4 * g + 3) * AW + mi]);
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
      int nj = cb * 16 + (lane & 15);
      float4 b = make_float4(Bs[(4 * g + 0) * BW + nj], Bs[(4 * g + 1) * BW + nj], Bs[(4 * g + 2) * BW + nj],
                             Bs[(4 * g + 3) * BW + nj]);
      mfma16<BF16>(a, b, acc[cb]);
    }
  }
  float* out = partial + (int64_t)blockIdx.y * M * N;
#pragma unroll
  for (int cb = 0; cb < NB; ++cb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int64_t m = m0 + wave * 16 + 4 * (lane >> 4) + r;
      int64_t nn = cb * 16 + (lane & 15);
      if (m < M && nn < N) out[m * N + nn] = acc[cb][r];
    }
}

__global__ void reduce_partials_kernel(const float* partial, int64_t nchunks, int64_t elems, double scale,
                                       double* out) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= elems) return;
  double acc = 0.0;
#pragma unroll 8
  for (int64_t c = 0; c < nchunks; ++c) acc += (double)partial[c * elems + e];
  out[e] = acc * scale;
}

// Column sums of the split-K partials, transposed: G[c ldg + j] = sum_chunk partial[chunk][j][c] (FP64, in
// chunk order), so that column c (one problem) becomes a contiguous row of G.
__global__ void reduce_partials_t_kernel(const float* partial, int64_t nchunks, int64_t d, int Pc, double* G,
                                         int64_t ldg) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t elems = d * Pc;
  if (e >= elems) return;
  double acc = 0.0;
#pragma unroll 8
  for (int64_t c = 0; c < nchunks; ++c) acc += (double)partial[c * elems + e];
  const int64_t j = e / Pc, col = e % Pc;
  G[col * ldg + j] = acc;
}

// R[i][p] -= Y[p mod ny][i] for the n x P residual matrix of a shared-X batch, and the FP64 residual
// sums of squares per (problem, row block): rsq[p nblk + blk].
__global__ __launch_bounds__(256) void residual_batched_kernel(float* R, int64_t n, int P, const float* Y, int ny,
                                                               int nblk, double* rsq) {
  const int64_t rows = (n + nblk - 1) / nblk;
  const int64_t i0 = (int64_t)blockIdx.x * rows;
  const int64_t i1 = i0 + rows < n ? i0 + rows : n;
  for (int c = threadIdx.x; c < P; c += blockDim.x) {
    const float* y = Y + (int64_t)(c % ny) * n;
    double acc = 0.0;
    for (int64_t i = i0; i < i1; ++i) {
      const float r = R[i * P + c] - y[i];
      R[i * P + c] = r;
      acc += (double)r * r;
    }
    rsq[(int64_t)c * nblk + blockIdx.x] = acc;
  }
}

bool aligned16(const void* p, int64_t ld) { return ((uintptr_t)p % 16 == 0) && (ld % 4 == 0); }

template <bool BF16>
int longk_dispatch(hipStream_t st, int nb, const float* A, int64_t M, int64_t K, int64_t lda, const float* Bt,
                   int64_t N, int64_t ldb, float* C, int64_t ldc) {
  dim3 grid((unsigned)cdiv(M, kLkBM));
  bool aa = aligned16(A, lda), ba = aligned16(Bt, ldb);
#define SCS_LK(NBV) \
  case NBV:         \
    gemm_nt_longk_kernel<NBV, BF16><<<grid, 256, 0, st>>>(A, M, K, lda, Bt, N, ldb, C, ldc, aa, ba); break;
  switch (nb) {
    SCS_LK(1) SCS_LK(2) SCS_LK(3) SCS_LK(4) SCS_LK(5) SCS_LK(6) SCS_LK(7) SCS_LK(8) SCS_LK(9)
    default:
      set_error("gemm_nt_longk: N > 144");
      return SCS_EINVAL;
  }
#undef SCS_LK
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

template <bool BF16>
int tn_dispatch(hipStream_t st, int nb, const float* A, int64_t R, int64_t M, int64_t lda, const float* B, int64_t N,
                int64_t ldb, float* partial, int64_t chunk_rows, int64_t nchunks) {
  dim3 grid((unsigned)cdiv(M, kTnBM), (unsigned)nchunks);
  bool aa = aligned16(A, lda), ba = aligned16(B, ldb);
#define SCS_TN(NBV)                                                                                             \
  case NBV:                                                                                                     \
    gemm_tn_splitk_kernel<NBV, BF16><<<grid, 256, 0, st>>>(A, R, M, lda, B, N, ldb, partial, chunk_rows, aa, \
                                                           ba);                                                 \
    break;
  switch (nb) {
    SCS_TN(1) SCS_TN(2) SCS_TN(3) SCS_TN(4) SCS_TN(5) SCS_TN(6) SCS_TN(7) SCS_TN(8) SCS_TN(9)
    default:
      set_error("gemm_tn_splitk: N > 144");
      return SCS_EINVAL;
  }
#undef SCS_TN
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

}  // namespace

int launch_gemm_nt_longk(hipStream_t st, int bf16, const float* A, int64_t M, int64_t K, int64_t lda,
                         const float* Bt, int64_t N, int64_t ldb, float* C, int64_t ldc) {
  if (M <= 0 || N <= 0) return SCS_OK;
  int nb = (int)cdiv(N, 16);
  return bf16 ? longk_dispatch<true>(st, nb, A, M, K, lda, Bt, N, ldb, C, ldc)
              : longk_dispatch<false>(st, nb, A, M, K, lda, Bt, N, ldb, C, ldc);
}

int launch_gemm_nt_wide(hipStream_t st, int bf16, const float* A, int64_t M, int64_t K, int64_t lda,
                        const float* Bt, int64_t N, int64_t ldb, float alpha, const float* C0, int64_t ldc0,
                        float beta, const double* beta_dev, float diag, const double* diag_dev, int out_bf16,
                        void* C, int64_t ldc, float* rownorm2) {
  if (M <= 0 || N <= 0) return SCS_OK;
  if (K > 160) {
    set_error("gemm_nt_wide: K > 160");
    return SCS_EINVAL;
  }
  int KP = (int)cdiv(K < 1 ? 1 : K, 16) * 16;
  size_t bytes = ((size_t)(kWdBM + kWdBN) * (KP + 4) + (size_t)kWdBM * (kWdBN + 4)) * sizeof(float);
  dim3 grid((unsigned)cdiv(M, kWdBM));
  bool aa = aligned16(A, lda), ba = aligned16(Bt, ldb);
  bool ca = C0 ? aligned16(C0, ldc0) : false;
  bool oa = out_bf16 ? ((uintptr_t)C % 8 == 0 && ldc % 4 == 0) : aligned16(C, ldc);
  const void* fn;
  if (bf16) fn = out_bf16 ? (const void*)gemm_nt_wide_kernel<true, true> : (const void*)gemm_nt_wide_kernel<true, false>;
  else fn = out_bf16 ? (const void*)gemm_nt_wide_kernel<false, true> : (const void*)gemm_nt_wide_kernel<false, false>;
  if (bytes > 65536) SCS_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
#define SCS_WD(B1, B2)                                                                                          \
  gemm_nt_wide_kernel<B1, B2><<<grid, 256, bytes, st>>>(A, M, K, lda, Bt, N, ldb, alpha, C0, ldc0, beta,     \
                                                         beta_dev, diag, diag_dev, C, ldc, rownorm2, KP, aa, ba, ca, oa)
  if (bf16) {
    if (out_bf16) SCS_WD(true, true);
    else SCS_WD(true, false);
  } else {
    if (out_bf16) SCS_WD(false, true);
    else SCS_WD(false, false);
  }
#undef SCS_WD
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_gemm_tn_splitk(hipStream_t st, int bf16, const float* A, int64_t R, int64_t M, int64_t lda,
                          const float* B, int64_t N, int64_t ldb, float* partial, int64_t chunk_rows,
                          int64_t nchunks) {
  if (M <= 0 || N <= 0) return SCS_OK;
  int nb = (int)cdiv(N, 16);
  return bf16 ? tn_dispatch<true>(st, nb, A, R, M, lda, B, N, ldb, partial, chunk_rows, nchunks)
              : tn_dispatch<false>(st, nb, A, R, M, lda, B, N, ldb, partial, chunk_rows, nchunks);
}

int launch_reduce_partials_t(hipStream_t st, const float* partial, int64_t nchunks, int64_t d, int Pc, double* G,
                             int64_t ldg) {
  if (d * Pc <= 0) return SCS_OK;
  reduce_partials_t_kernel<<<dim3((unsigned)cdiv(d * Pc, 256)), dim3(256), 0, st>>>(partial, nchunks, d, Pc, G, ldg);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_residual_batched(hipStream_t st, float* R, int64_t n, int P, const float* Y, int ny, int nblk,
                            double* rsq) {
  if (n <= 0 || P <= 0) return SCS_OK;
  residual_batched_kernel<<<dim3((unsigned)nblk), dim3(256), 0, st>>>(R, n, P, Y, ny, nblk, rsq);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_reduce_partials_f64(hipStream_t st, const float* partial, int64_t nchunks, int64_t elems, double scale,
                               double* out) {
  if (elems <= 0) return SCS_OK;
  reduce_partials_kernel<<<dim3((unsigned)cdiv(elems, 256)), dim3(256), 0, st>>>(partial, nchunks, elems, scale,
                                                                                 out);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

}  // namespace scs
