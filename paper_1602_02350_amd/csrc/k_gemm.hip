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
#include <map>
#include <mutex>
#include <tuple>

#include "scs_internal.h"

namespace scs {

namespace {

// Workgroups of `fn` that fit on the current device at once (cached per kernel, LDS size and
// device); 0 when the runtime cannot say.
int resident_blocks(const void* fn, int threads, size_t lds) {
  static std::mutex mu;
  static std::map<std::tuple<const void*, size_t, int>, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  std::lock_guard<std::mutex> lk(mu);
  const auto key = std::make_tuple(fn, lds, dev);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  const int r = per_cu * cus;
  cache[key] = r;
  return r;
}

typedef float f4v __attribute__((ext_vector_type(4)));
typedef short s4v __attribute__((ext_vector_type(4)));
typedef short s8v __attribute__((ext_vector_type(8)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

// gfx950's 16x16x32 BF16 MFMA. Lane (r, g) supplies 8 K values of row (A) or column (B) r; the kernels
// give it the 4-value fragments of two consecutive 16-wide K blocks (K 16 q + 4 g .. +3 and
// 16 (q + 1) + 4 g .. +3) in both operands, so every product pairs equal K and the 32 K values of the
// two blocks are each summed once.
__device__ __forceinline__ s8v cat8(const s4v& lo, const s4v& hi) {
  return __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
}
__device__ __forceinline__ f4v mfma_bf16_k32(const s8v& a, const s8v& b, const f4v& acc) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8v, a), __builtin_bit_cast(bf8v, b), acc, 0,
                                                 0, 0);
}

__device__ __forceinline__ short bf16s(float f) { return (short)f32_to_bf16(f); }
__device__ __forceinline__ s4v bf16x4(const float4& a) { return s4v{bf16s(a.x), bf16s(a.y), bf16s(a.z), bf16s(a.w)}; }

__device__ __forceinline__ bool gate_shut(const Gate& g) { return g.count && *g.count >= g.total; }

// four FP32 16x16x4 MFMAs over the K values a.x .. a.w (lane (r, g): K 4 g .. 4 g + 3 of a 16-wide block)
__device__ __forceinline__ void mfma16_f32(const float4& a, const float4& b, f4v& acc) {
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b.z, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b.w, acc, 0, 0, 0);
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
                                                            int64_t nst, bool a_al, bool b_al, Gate gate) {
  if (gate_shut(gate)) return;
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
    if constexpr (BF16) {
      static_assert(kLkBK == 32, "one 16x16x32 MFMA per chunk");
      const int ko = 4 * (lane >> 4);
      const float* a0p = &As[(wave * 32 + (lane & 15)) * LDS_W + ko];
      const float* a1p = &As[(wave * 32 + 16 + (lane & 15)) * LDS_W + ko];
      const s8v a0 = cat8(bf16x4(*reinterpret_cast<const float4*>(a0p)),
                          bf16x4(*reinterpret_cast<const float4*>(a0p + 16)));
      const s8v a1 = cat8(bf16x4(*reinterpret_cast<const float4*>(a1p)),
                          bf16x4(*reinterpret_cast<const float4*>(a1p + 16)));
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) {
        const float* bp = &Bs[(cb * 16 + (lane & 15)) * LDS_W + ko];
        const s8v b = cat8(bf16x4(*reinterpret_cast<const float4*>(bp)),
                           bf16x4(*reinterpret_cast<const float4*>(bp + 16)));
        acc[0][cb] = mfma_bf16_k32(a0, b, acc[0][cb]);
        acc[1][cb] = mfma_bf16_k32(a1, b, acc[1][cb]);
      }
    } else {
#pragma unroll
      for (int kq = 0; kq < kLkBK; kq += 16) {
        const int ko = kq + 4 * (lane >> 4);
        float4 a0 = *reinterpret_cast<const float4*>(&As[(wave * 32 + (lane & 15)) * LDS_W + ko]);
        float4 a1 = *reinterpret_cast<const float4*>(&As[(wave * 32 + 16 + (lane & 15)) * LDS_W + ko]);
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) {
          float4 b = *reinterpret_cast<const float4*>(&Bs[(cb * 16 + (lane & 15)) * LDS_W + ko]);
          mfma16_f32(a0, b, acc[0][cb]);
          mfma16_f32(a1, b, acc[1][cb]);
        }
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
        if (row < M && col < nst) C[row * ldc + col] = acc[rbk][cb][r];
      }
}

// ------------------------------------------------------------------ narrow Gram W^T W (FP32)
// Partial Gram matrices of W (R x L row-major, leading dimension ldw, L <= 64): workgroup g sums rows
// [g chunk, (g + 1) chunk) in 64-row slabs staged transposed in LDS (Ws[c][r]); wave w owns output rows
// 16 w .. 16 w + 15 and all four 16-column blocks, with the FP32 16x16x4 MFMA over the slab's rows
// (lane (r, q) feeds rows 4 q .. 4 q + 3 of each group of 16, as mfma16_f32 takes them).
// partial[g][i L + j] = sum over the chunk of W[r][i] W[r][j] (i, j < L).
constexpr int kGramSlab = 64;
constexpr int kGramLW = kGramSlab + 4;  // LDS row pitch of the transposed slab (floats)

__global__ __launch_bounds__(256) void gram_rr_f32_kernel(const float* __restrict__ W, int64_t R, int L, int64_t ldw,
                                                          int64_t chunk, float* __restrict__ partial) {
  __shared__ __align__(16) float Ws[64 * kGramLW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t r_begin = (int64_t)blockIdx.x * chunk;
  const int64_t r_end = r_begin + chunk < R ? r_begin + chunk : R;
  f4v acc[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) acc[cb] = f4v{0.f, 0.f, 0.f, 0.f};
  // Thread tid stages rows (tid >> 6) + 4 q, column c = tid & 63 of each slab. Loads are unconditional
  // from a clamped address (row and column inside W) and masked to zero when stored to LDS, so the 16
  // loads of a slab are in flight together; the next slab is loaded while the MFMAs consume this one.
  const int c = tid & 63, rr = tid >> 6;
  const bool col_ok = c < L;
  const int cc = col_ok ? c : L - 1;
  float v[16];
  auto load_slab = [&](int64_t r0) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int64_t row = r0 + rr + 4 * q;
      const int64_t rc = row < r_end ? row : r_end - 1;
      v[q] = W[rc * ldw + cc];
    }
  };
  load_slab(r_begin);
  for (int64_t r0 = r_begin; r0 < r_end; r0 += kGramSlab) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) Ws[c * kGramLW + rr + 4 * q] = (col_ok && r0 + rr + 4 * q < r_end) ? v[q] : 0.f;
    __syncthreads();
    if (r0 + kGramSlab < r_end) load_slab(r0 + kGramSlab);
#pragma unroll
    for (int kq = 0; kq < kGramSlab; kq += 16) {
      const int ko = kq + 4 * (lane >> 4);
      const float4 a = *reinterpret_cast<const float4*>(&Ws[(wave * 16 + (lane & 15)) * kGramLW + ko]);
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        const float4 b = *reinterpret_cast<const float4*>(&Ws[(cb * 16 + (lane & 15)) * kGramLW + ko]);
        mfma16_f32(a, b, acc[cb]);
      }
    }
  }
  float* out = partial + (int64_t)blockIdx.x * L * L;
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = wave * 16 + 4 * (lane >> 4) + r, j = cb * 16 + (lane & 15);
      if (i < L && j < L) out[(int64_t)i * L + j] = acc[cb][r];
    }
}

// ------------------------------------------------------------------ NT, long K, A in registers
// The same product as gemm_nt_longk for 16-byte aligned rows of A (X): each wave owns 16 rows of A
// and reads its MFMA fragments straight from global memory into registers, one K chunk ahead
// (lane (r, g) holds A[row0 + r][k0 + 16 q + 4 g .. +3] in FP32, A[row0 + r][k0 + 32 p + 8 g .. +7] for
// the BF16 16x16x32 MFMA); Bt's K chunk (N <= 144 rows) is staged
// through LDS, double-buffered and rounded to BF16 once in BF16 mode. One barrier per chunk;
// workgroups loop over row tiles (grid sized to the resident capacity). The last chunk, where K may
// end inside it, is loaded with guards.
// BF16: 512 threads (128-row tiles), four waves per SIMD; FP32: 256 threads (64-row tiles), three waves
// per SIMD. Timed at n = 100000, K = 1000, N = 55 (FP32): 190 -> 172 us; at n = 500000, K = 2048,
// N = 133 (BF16) the 512-thread kernel stays fastest (1170 us against 1280-1350 us for 256 threads or
// two waves per SIMD, although it spills some registers there).
constexpr int lr_threads(bool bf16) { return bf16 ? 512 : 256; }
constexpr int lr_waves(bool bf16) { return bf16 ? 4 : 3; }

template <int NB, bool BF16>
__global__ __launch_bounds__(lr_threads(BF16), lr_waves(BF16)) void gemm_nt_longk_reg_kernel(
    const float* __restrict__ A, int64_t M, int64_t K, int64_t lda, const float* __restrict__ Bt, int64_t N,
    int64_t ldb, float* __restrict__ C, int64_t ldc, int64_t nst, Gate gate) {
  if (gate_shut(gate)) return;
  constexpr int KC = BF16 ? 64 : 32;          // K per chunk
  constexpr int kLrThreads = lr_threads(BF16), kLrBM = 16 * (kLrThreads / 64);
  constexpr int NQ = KC / 16;                  // MFMA K steps per chunk
  constexpr int BN = NB * 16;
  constexpr int LW = KC + 4, LH = KC + 8;      // LDS row strides (floats / BF16 halves)
  constexpr int BUF = BF16 ? BN * LH / 2 : BN * LW;
  constexpr int NE = BN * (KC / 4);            // float4 per Bt chunk
  constexpr int RB = (NE + kLrThreads - 1) / kLrThreads;
  __shared__ float S[2 * BUF];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rl = lane & 15, g4 = 4 * (lane >> 4);
  const int64_t nch = (K + KC - 1) / KC;
  const int64_t ntiles = (M + kLrBM - 1) / kLrBM;

  f4v rb[RB];
  auto load_b = [&](int64_t c) {
    const int64_t k0 = c * KC;
#pragma unroll
    for (int j = 0; j < RB; ++j) {
      const int e = tid + kLrThreads * j;
      const int r = e / (KC / 4), c4 = e % (KC / 4);
      const int64_t k = k0 + 4 * c4;
      f4v v = {0.f, 0.f, 0.f, 0.f};
      if (e < NE && r < N) {
        const float* p = Bt + (int64_t)r * ldb + k;
        if (k + 3 < K) {
          v[0] = p[0];
          v[1] = p[1];
          v[2] = p[2];
          v[3] = p[3];
        } else {
          if (k < K) v[0] = p[0];
          if (k + 1 < K) v[1] = p[1];
          if (k + 2 < K) v[2] = p[2];
        }
      }
      rb[j] = v;
    }
  };
  auto stash_b = [&](int bsel) {
    float* base = S + bsel * BUF;
#pragma unroll
    for (int j = 0; j < RB; ++j) {
      const int e = tid + kLrThreads * j;
      if (e < NE) {
        const int r = e / (KC / 4), c4 = e % (KC / 4);
        if constexpr (BF16) {
          *reinterpret_cast<uint2*>(reinterpret_cast<uint16_t*>(base) + r * LH + 4 * c4) =
              make_uint2(pack_bf16x2(rb[j][0], rb[j][1]), pack_bf16x2(rb[j][2], rb[j][3]));
        } else {
          *reinterpret_cast<f4v*>(base + r * LW + 4 * c4) = rb[j];
        }
      }
    }
  };

  // K offset of fragment q within a chunk: FP32 lane group g takes K 16 q + 4 g .. +3; BF16 lane group g
  // takes the 8 consecutive K 32 (q / 2) + 8 g .. +7 of the 16x16x32 MFMA, as fragments q (even) and q + 1
  const int ga = BF16 ? 2 * g4 : g4;
  auto koff = [](int q) { return BF16 ? 32 * (q >> 1) + 4 * (q & 1) : 16 * q; };
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t row = tile * kLrBM + wave * 16 + rl;
    const float* arow = A + (row < M ? row : M - 1) * lda + ga;
    f4v af[NQ], an[NQ];   // chunks c and c + 1
    auto load_a = [&](int64_t c, f4v (&dst)[NQ]) {
      const int64_t k0 = c * KC;
      if (k0 + KC <= K) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) dst[q] = *reinterpret_cast<const f4v*>(arow + k0 + koff(q));
      } else {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const int64_t k = k0 + koff(q) + ga;
          f4v v = {0.f, 0.f, 0.f, 0.f};
          if (k + 3 < K) {
            v = *reinterpret_cast<const f4v*>(arow + k0 + koff(q));
          } else {
            const float* p = arow + k0 + koff(q);
            if (k < K) v[0] = p[0];
            if (k + 1 < K) v[1] = p[1];
            if (k + 2 < K) v[2] = p[2];
          }
          dst[q] = v;
        }
      }
    };
    f4v acc[NB];
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) acc[cb] = f4v{0.f, 0.f, 0.f, 0.f};

    __syncthreads();   // the previous tile's chunk buffers are free
    load_b(0);
    stash_b(0);
    if (nch > 1) load_b(1);
    load_a(0, af);
    __syncthreads();
    for (int64_t c = 0; c < nch; ++c) {
      if (c + 1 < nch) load_a(c + 1, an);
      const float* base = S + (int)(c & 1) * BUF;
#pragma unroll
      for (int q = 0; q < NQ; q += BF16 ? 2 : 1) {
        if constexpr (BF16) {
          static_assert(NQ % 2 == 0, "K blocks are taken in pairs");
          const uint32_t l0 = pack_bf16x2(af[q][0], af[q][1]), h0 = pack_bf16x2(af[q][2], af[q][3]);
          const uint32_t l1 = pack_bf16x2(af[q + 1][0], af[q + 1][1]), h1 = pack_bf16x2(af[q + 1][2], af[q + 1][3]);
          const s8v ah = {(short)(l0 & 0xffff), (short)(l0 >> 16), (short)(h0 & 0xffff), (short)(h0 >> 16),
                          (short)(l1 & 0xffff), (short)(l1 >> 16), (short)(h1 & 0xffff), (short)(h1 >> 16)};
#pragma unroll
          for (int cb = 0; cb < NB; ++cb) {
            const s8v bv = *reinterpret_cast<const s8v*>(reinterpret_cast<const uint16_t*>(base) +
                                                         (cb * 16 + rl) * LH + 16 * q + ga);
            acc[cb] = mfma_bf16_k32(ah, bv, acc[cb]);
          }
        } else {
#pragma unroll
          for (int cb = 0; cb < NB; ++cb) {
            const f4v bv = *reinterpret_cast<const f4v*>(base + (cb * 16 + rl) * LW + 16 * q + g4);
            acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[q][0], bv[0], acc[cb], 0, 0, 0);
            acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[q][1], bv[1], acc[cb], 0, 0, 0);
            acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[q][2], bv[2], acc[cb], 0, 0, 0);
            acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[q][3], bv[3], acc[cb], 0, 0, 0);
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      if (c + 1 < nch) {
        stash_b((int)((c + 1) & 1));
        if (c + 2 < nch) load_b(c + 2);
#pragma unroll
        for (int q = 0; q < NQ; ++q) af[q] = an[q];
      }
      __syncthreads();
    }
    // acc[cb][r] = C[row0 + 4 (lane / 16) + r][16 cb + lane % 16]
    const int64_t r0 = tile * kLrBM + wave * 16 + g4;
#pragma unroll
    for (int cb = 0; cb < NB; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t rr = r0 + r;
        const int64_t cc = cb * 16 + rl;
        if (rr < M && cc < nst) C[rr * ldc + cc] = acc[cb][r];
      }
  }
}

// ------------------------------------------------------------------ TN split-K, A in registers
// partial[chunk] = A[rows of chunk]^T B[rows of chunk] for 16-byte aligned rows of A and B (M x N per
// chunk, row-major). Wave w owns 16 TC columns of A (TC = 4 for N <= 64, else 2), starting at
// m_base = blockIdx.x 8 16 TC + 16 TC w. Lane (r, g) loads A[row][m_base + TC r .. + TC - 1] as one
// vector (16 lanes cover 16 TC contiguous floats of a row, 4 rows per instruction), and component c
// of it feeds output tile c: rows m = m_base + TC i + c. With the FP32 16x16x4 MFMA a K step is 4
// rows (lane group g supplies row g); with gfx950's BF16 16x16x32 MFMA a K step is 32 rows (lane group g
// supplies rows 8 g .. 8 g + 7, from eight loads). B's rows are staged through LDS in tiles of 64
// rows, double-buffered (FP32 row-major; BF16 transposed and rounded once), one barrier per tile;
// the A loads of the next K step are issued before the MFMAs of the current one.
constexpr int kTgThreads = 512;
constexpr int tg_tc(int nb) { return nb <= 4 ? 4 : 2; }
constexpr int tg_cols(int nb) { return (kTgThreads / 64) * 16 * tg_tc(nb); }  // columns of A per workgroup

template <int NB, bool BF16>
__global__ __launch_bounds__(kTgThreads) void gemm_tn_reg_kernel(const float* __restrict__ A, int64_t R, int64_t M,
                                                                 int64_t lda, const float* __restrict__ B, int64_t N,
                                                                 int64_t ldb, float* __restrict__ partial,
                                                                 int64_t chunk_rows, Gate gate) {
  if (gate_shut(gate)) return;
  constexpr int TC = tg_tc(NB);                // output tiles (columns of A per lane)
  constexpr int KS = BF16 ? 32 : 4;            // rows per K step
  constexpr int KR = 64;                       // rows per staged B tile
  constexpr int SPT = KR / KS;                 // K steps per tile
  constexpr int BN = NB * 16;
  constexpr int LF = BN + 4;                   // FP32 tile: [KR][LF] floats
  constexpr int LH = KR + 8;                   // BF16 tile: [BN][LH] halves (transposed)
  constexpr int BUF = BF16 ? BN * LH / 2 : KR * LF;
  constexpr int NE = KR * BN / 4;              // float4 per B tile
  constexpr int RB = (NE + kTgThreads - 1) / kTgThreads;
  constexpr int NL = BF16 ? 8 : 1;             // loads of A per lane and K step
  typedef float tcv __attribute__((ext_vector_type(TC)));
  __shared__ float S[2 * BUF];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int rl = lane & 15, g = lane >> 4;
  const int64_t m_base = (int64_t)blockIdx.x * tg_cols(NB) + 16 * TC * wave;
  const int64_t r0 = (int64_t)blockIdx.y * chunk_rows;
  const int64_t r1 = r0 + chunk_rows < R ? r0 + chunk_rows : R;
  const int64_t nrows = r1 > r0 ? r1 - r0 : 0;
  const int64_t ntile = (nrows + KR - 1) / KR;
  const int64_t mcol = m_base + TC * rl;        // this lane's first column of A
  const bool wave_on = m_base < M;              // uniform

  f4v rbuf[RB];
  auto load_b = [&](int64_t t) {
#pragma unroll
    for (int j = 0; j < RB; ++j) {
      const int e = tid + kTgThreads * j;
      const int r = e / (BN / 4), c4 = e % (BN / 4);
      const int64_t row = r0 + t * KR + r;
      const int64_t n = 4 * c4;
      f4v v = {0.f, 0.f, 0.f, 0.f};
      if (e < NE && row < r1) {
        const float* p = B + row * ldb + n;
        if (n + 3 < N) {
          v = *reinterpret_cast<const f4v*>(p);
        } else {
          if (n < N) v[0] = p[0];
          if (n + 1 < N) v[1] = p[1];
          if (n + 2 < N) v[2] = p[2];
        }
      }
      rbuf[j] = v;
    }
  };
  auto stash_b = [&](int bsel) {
    float* base = S + bsel * BUF;
#pragma unroll
    for (int j = 0; j < RB; ++j) {
      const int e = tid + kTgThreads * j;
      if (e < NE) {
        const int r = e / (BN / 4), c4 = e % (BN / 4);
        if constexpr (BF16) {
          uint16_t* h = reinterpret_cast<uint16_t*>(base);
#pragma unroll
          for (int v = 0; v < 4; ++v) h[(4 * c4 + v) * LH + r] = f32_to_bf16(rbuf[j][v]);
        } else {
          *reinterpret_cast<f4v*>(base + r * LF + 4 * c4) = rbuf[j];
        }
      }
    }
  };
  // A rows of K step s (global step index) for this lane
  auto load_a = [&](int64_t s, tcv (&x)[NL]) {
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int64_t row = r0 + s * KS + (BF16 ? 8 * g + u : g);
      tcv v;
#pragma unroll
      for (int c = 0; c < TC; ++c) v[c] = 0.f;
      if (wave_on && row < r1) {
        const float* p = A + row * lda + mcol;
        if (mcol + TC - 1 < M) {
          v = *reinterpret_cast<const tcv*>(p);
        } else {
#pragma unroll
          for (int c = 0; c < TC; ++c)
            if (mcol + c < M) v[c] = p[c];
        }
      }
      x[u] = v;
    }
  };

  f4v acc[TC][NB];
#pragma unroll
  for (int c = 0; c < TC; ++c)
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) acc[c][cb] = f4v{0.f, 0.f, 0.f, 0.f};

  const int64_t nsteps = ntile * SPT;
  tcv xa[NL], xn[NL];
  if (ntile > 0) {
    load_b(0);
    stash_b(0);
    if (ntile > 1) load_b(1);
    load_a(0, xa);
  }
  __syncthreads();
  for (int64_t t = 0; t < ntile; ++t) {
    const float* base = S + (int)(t & 1) * BUF;
#pragma unroll
    for (int ss = 0; ss < SPT; ++ss) {
      const int64_t s = t * SPT + ss;
      if (s + 1 < nsteps) load_a(s + 1, xn);
      if (wave_on) {
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) {
          if constexpr (BF16) {
            const s8v bv = *reinterpret_cast<const s8v*>(reinterpret_cast<const uint16_t*>(base) +
                                                         (16 * cb + rl) * LH + ss * KS + 8 * g);
#pragma unroll
            for (int c = 0; c < TC; ++c) {
              s8v av;
#pragma unroll
              for (int u = 0; u < 8; u += 2) {
                const uint32_t h = pack_bf16x2(xa[u][c], xa[u + 1][c]);
                av[u] = (short)(h & 0xffff);
                av[u + 1] = (short)(h >> 16);
              }
              acc[c][cb] = mfma_bf16_k32(av, bv, acc[c][cb]);
            }
          } else {
            const float bv = base[(ss * KS + g) * LF + 16 * cb + rl];
#pragma unroll
            for (int c = 0; c < TC; ++c)
              acc[c][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[0][c], bv, acc[c][cb], 0, 0, 0);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < NL; ++u) xa[u] = xn[u];
    }
    if (t + 1 < ntile) {
      stash_b((int)((t + 1) & 1));
      if (t + 2 < ntile) load_b(t + 2);
    }
    __syncthreads();
  }
  // acc[c][cb][r] = out[m_base + TC (4 (lane / 16) + r) + c][16 cb + lane % 16]
  if (!wave_on) return;
  float* out = partial + (int64_t)blockIdx.y * M * N;
#pragma unroll
  for (int c = 0; c < TC; ++c)
#pragma unroll
    for (int cb = 0; cb < NB; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = m_base + TC * (4 * g + r) + c;
        const int64_t n = 16 * cb + rl;
        if (m < M && n < N) out[m * N + n] = acc[c][cb][r];
      }
}

// ------------------------------------------------------------------ NT, wide N, short K
// C = alpha A Bt^T + beta C0 (+ diag where row == col). A is M x KP and Bt is (N rounded up to 64) x KP
// with KP = gemm_wide_kpad(K) (16, 32, 64, 128 or 160). Bt is zero past K and past N; A is zero from K
// to the next multiple of 16 and its 16-column blocks past that are ignored. The only load that needs
// a guard is A's row, clamped once per tile. The MFMA runs transposed, D = Bt_chunk A^T, so
// that acc[r] = C[row0 + lane % 16][col0 + 4 (lane / 16) + r]: each lane ends with four consecutive
// columns of one row. In the vector path (N % 4 == 0) lanes rl and rl ^ 8 then swap one block of each
// pair of 16-column blocks, so that every C0 load and C store covers 8 rows x 32 columns (128 contiguous
// bytes per row in FP32) instead of 16 rows x 16 columns; the epilogue reads C0 and writes C with
// 16-byte (8-byte for BF16) accesses straight from registers. Each wave owns 16 rows whose A fragments
// stay in registers for the whole tile; Bt is streamed through LDS in 64-row chunks, double-buffered
// (rounded to BF16 once at staging in BF16 mode), and C0 is fetched one chunk ahead (two for K = 64).
// Workgroups loop over row tiles (grid sized to the resident capacity).
// K <= 64: 512 threads (128-row tiles); wider K holds more A fragments per lane: 256 threads (64-row
// tiles). Four waves per SIMD for K <= 32, else two. Timed on the apply shapes (n = 100000, d = 1000,
// K = 50, FP32; n = 500000, d = 2048, K = 128, BF16): 300 -> 279 us and 1870 -> 1597 us against the
// unswapped epilogue with one chunk ahead and four or three waves (where K = 128 spilled registers).
constexpr int wd_threads(int nkq) { return nkq <= 4 ? 512 : 256; }
constexpr int wd_waves(int nkq) { return nkq <= 2 ? 4 : 2; }
constexpr int wd_ahead(int nkq) { return nkq == 4 ? 2 : 1; }   // C0 chunks fetched ahead
constexpr int kWdBN = 64;                       // output columns per chunk

template <bool BF16, bool OUT_BF16, int NKQ, bool VEC>
__global__ __launch_bounds__(wd_threads(NKQ), wd_waves(NKQ)) void gemm_nt_wide_kernel(
    const float* __restrict__ A, int64_t M, int64_t lda, const float* __restrict__ Bt, int N, int64_t ldb,
    float alpha, const float* __restrict__ C0, int64_t ldc0, float beta, const double* beta_dev, float diag,
    const double* diag_dev, void* Cout, int64_t ldc, float* __restrict__ rownorm2, int nq) {
  extern __shared__ float S[];
  constexpr int KP = 16 * NKQ;                 // A blocks q >= nq (K rounded up to 16, over 16) count as zero
  constexpr int LW = KP + 4, LH = KP + 8;      // LDS row strides: floats, BF16 halves
  constexpr int BUF = BF16 ? kWdBN * LH / 2 : kWdBN * LW;
  constexpr int kWdThreads = wd_threads(NKQ);
  constexpr int kWdBM = 16 * (kWdThreads / 64);   // rows per tile: 16 per wave
  constexpr int RB = (kWdBN * 4 * NKQ + kWdThreads - 1) / kWdThreads;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rl = lane & 15, g4 = 4 * (lane >> 4);
  constexpr int kv = 4 * NKQ;                  // float4 per Bt row
  constexpr int ne = kWdBN * kv;               // float4 per chunk
  const int nch = (N + kWdBN - 1) / kWdBN;
  const int64_t ntiles = (M + kWdBM - 1) / kWdBM;
  if (beta_dev) beta = (float)beta_dev[0];
  if (diag_dev) diag = (float)diag_dev[0];

  // staging slot j of this thread: float4 e = tid + threads j of the chunk, row e / kv, column 4 (e % kv);
  // a slot past the chunk re-reads the chunk's first float4 and is not stored
  f4v rb[RB];
  auto load_b = [&](int c) {
    const float* base = Bt + (int64_t)c * kWdBN * ldb;
#pragma unroll
    for (int j = 0; j < RB; ++j) {
      const int e = tid + kWdThreads * j;
      const int off = (ne % kWdThreads == 0 || e < ne) ? (e / kv) * (int)ldb + 4 * (e % kv) : 0;
      rb[j] = *reinterpret_cast<const f4v*>(base + off);
    }
  };
  auto stash_b = [&](int bsel) {
    float* base = S + bsel * BUF;
#pragma unroll
    for (int j = 0; j < RB; ++j) {
      const int e = tid + kWdThreads * j;
      if (ne % kWdThreads == 0 || e < ne) {
        const int r = e / kv, c4 = e % kv;
        if constexpr (BF16) {
          const uint2 h = make_uint2(pack_bf16x2(rb[j][0], rb[j][1]), pack_bf16x2(rb[j][2], rb[j][3]));
          *reinterpret_cast<uint2*>(reinterpret_cast<uint16_t*>(base) + r * LH + 4 * c4) = h;
        } else {
          *reinterpret_cast<f4v*>(base + r * LW + 4 * c4) = rb[j];
        }
      }
    }
  };

  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t row = tile * kWdBM + wave * 16 + rl;
    const bool row_ok = row < M;
    const int64_t rowc = row_ok ? row : M - 1;
    // A fragments: lane holds A[row][16 q + g4 .. +3] (FP32, or BF16 with an odd block count), or for
    // the BF16 16x16x32 MFMA the 8 consecutive A[row][32 (q / 2) + 2 g4 .. +7] as fragments q and q + 1
    constexpr bool K32 = BF16 && NKQ % 2 == 0;
    const int ga = K32 ? 2 * g4 : g4;
    auto koff = [](int q) { return K32 ? 32 * (q >> 1) + 4 * (q & 1) : 16 * q; };
    float4 af[NKQ];
    s4v ah[NKQ];
    {
      const float* arow = A + rowc * lda + ga;
#pragma unroll
      for (int q = 0; q < NKQ; ++q) {
        float4 v = *reinterpret_cast<const float4*>(arow + koff(q));
        if (koff(q) + ga >= 16 * nq) v = make_float4(0.f, 0.f, 0.f, 0.f);   // past the valid 16-column blocks
        if constexpr (BF16) {
          const uint32_t lo = pack_bf16x2(v.x, v.y), hi = pack_bf16x2(v.z, v.w);
          ah[q] = s4v{(short)(lo & 0xffff), (short)(lo >> 16), (short)(hi & 0xffff), (short)(hi >> 16)};
        } else {
          af[q] = v;
        }
      }
    }
    // vector path: lane (rl, g4) handles rows rA = rl & 7 and rA + 8 of the wave's 16, at column quad
    // 16 (2 p + (rl >= 8)) + g4 of each 32-column pair p of the chunk
    const bool lo8 = rl < 8;
    const int64_t rowA = tile * kWdBM + wave * 16 + (rl & 7), rowB = rowA + 8;
    const float* xrow = C0 ? C0 + rowc * ldc0 : nullptr;
    const float* xrowA = C0 ? C0 + (rowA < M ? rowA : M - 1) * ldc0 : nullptr;
    const float* xrowB = C0 ? C0 + (rowB < M ? rowB : M - 1) * ldc0 : nullptr;
    constexpr int AHEAD = wd_ahead(NKQ);
    float4 xc0[4], xc1[4];
    auto load_x = [&](int c, float4 (&xd)[4]) {
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        if (!xrow) {
          xd[cb] = make_float4(0.f, 0.f, 0.f, 0.f);
        } else if constexpr (VEC) {
          const int col = c * kWdBN + (2 * (cb >> 1) + (lo8 ? 0 : 1)) * 16 + g4;
          xd[cb] = *reinterpret_cast<const float4*>(((cb & 1) ? xrowB : xrowA) + min(col, N - 4));
        } else {
          const int col = c * kWdBN + cb * 16 + g4;
          xd[cb] = make_float4(xrow[min(col, N - 1)], xrow[min(col + 1, N - 1)], xrow[min(col + 2, N - 1)],
                               xrow[min(col + 3, N - 1)]);
        }
      }
    };
    // v = alpha acc + beta x (+ diag), rounded to BF16 in BF16 output mode; stored when in range, with
    // its squares added to r
    auto emit = [&](const f4v& a, const float4& x, int64_t rw, int col, float& r) {
      float v[4] = {alpha * a[0], alpha * a[1], alpha * a[2], alpha * a[3]};
      if (xrow) {
        v[0] = fmaf(beta, x.x, v[0]);
        v[1] = fmaf(beta, x.y, v[1]);
        v[2] = fmaf(beta, x.z, v[2]);
        v[3] = fmaf(beta, x.w, v[3]);
      }
      if (diag != 0.f) {
        const int64_t dq = rw - col;   // v[dq] sits on the diagonal when 0 <= dq < 4
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (dq == q) v[q] += diag;
      }
      uint32_t lo = 0, hi = 0;
      if constexpr (OUT_BF16) {
        lo = pack_bf16x2(v[0], v[1]);
        hi = pack_bf16x2(v[2], v[3]);
        v[0] = __uint_as_float(lo << 16);
        v[1] = __uint_as_float(lo & 0xffff0000u);
        v[2] = __uint_as_float(hi << 16);
        v[3] = __uint_as_float(hi & 0xffff0000u);
      }
      if (rw >= M || col >= N) return;
      if constexpr (VEC) {
        if constexpr (OUT_BF16)
          *reinterpret_cast<uint2*>(reinterpret_cast<uint16_t*>(Cout) + rw * ldc + col) = make_uint2(lo, hi);
        else
          *reinterpret_cast<float4*>(reinterpret_cast<float*>(Cout) + rw * ldc + col) =
              make_float4(v[0], v[1], v[2], v[3]);
        r = fmaf(v[0], v[0], r);
        r = fmaf(v[1], v[1], r);
        r = fmaf(v[2], v[2], r);
        r = fmaf(v[3], v[3], r);
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (col + q < N) {
            if constexpr (OUT_BF16)
              reinterpret_cast<uint16_t*>(Cout)[rw * ldc + col + q] = (uint16_t)((q < 2 ? lo : hi) >> (16 * (q & 1)));
            else
              reinterpret_cast<float*>(Cout)[rw * ldc + col + q] = v[q];
            r = fmaf(v[q], v[q], r);
          }
        }
      }
    };
    float rn = 0.f, rn1 = 0.f;   // squares of rows rowA and rowB (vector path), of row (else rn)

    __syncthreads();   // the previous tile's chunk buffers are free
    load_b(0);
    stash_b(0);
    if (nch > 1) load_b(1);
    load_x(0, xc0);
    if (AHEAD == 2 && nch > 1) load_x(1, xc1);
    __syncthreads();
    auto chunk = [&](int c, float4 (&xcur)[4]) {
      f4v acc[4];
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) acc[cb] = f4v{0.f, 0.f, 0.f, 0.f};
      const float* base = S + (c & 1) * BUF;
#pragma unroll
      for (int q = 0; q < NKQ; q += K32 ? 2 : 1) {
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
          if constexpr (K32) {
            const s8v bv = *reinterpret_cast<const s8v*>(reinterpret_cast<const uint16_t*>(base) + (cb * 16 + rl) * LH +
                                                         16 * q + ga);
            acc[cb] = mfma_bf16_k32(bv, cat8(ah[q], ah[q + 1]), acc[cb]);
          } else if constexpr (BF16) {   // one 16-wide K block (K = 16)
            const s4v bv = *reinterpret_cast<const s4v*>(reinterpret_cast<const uint16_t*>(base) + (cb * 16 + rl) * LH +
                                                         16 * q + g4);
            acc[cb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(bv, ah[q], acc[cb], 0, 0, 0);
          } else {
            const float4 bv = *reinterpret_cast<const float4*>(base + (cb * 16 + rl) * LW + 16 * q + g4);
            acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(bv.x, af[q].x, acc[cb], 0, 0, 0);
            acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(bv.y, af[q].y, acc[cb], 0, 0, 0);
            acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(bv.z, af[q].z, acc[cb], 0, 0, 0);
            acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(bv.w, af[q].w, acc[cb], 0, 0, 0);
          }
        }
        __builtin_amdgcn_sched_barrier(0);   // keeps each step's LDS reads next to their MFMAs
      }
      if (c + 1 < nch) {
        stash_b((c + 1) & 1);
        if (c + 2 < nch) load_b(c + 2);
      }
      // epilogue
      if constexpr (VEC) {
#pragma unroll
        for (int pr = 0; pr < 2; ++pr) {
          // the low lanes keep block 2 pr and receive the high lanes' block 2 pr (rows rA + 8); the high
          // lanes keep block 2 pr + 1 and receive the low lanes' block 2 pr + 1 (rows rA)
          const f4v snd = lo8 ? acc[2 * pr + 1] : acc[2 * pr];
          f4v rcv;
#pragma unroll
          for (int i = 0; i < 4; ++i) rcv[i] = __shfl_xor(snd[i], 8);
          const int col = c * kWdBN + (2 * pr + (lo8 ? 0 : 1)) * 16 + g4;
          emit(lo8 ? acc[2 * pr] : rcv, xcur[2 * pr], rowA, col, rn);
          emit(lo8 ? rcv : acc[2 * pr + 1], xcur[2 * pr + 1], rowB, col, rn1);
        }
      } else {
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) emit(acc[cb], xcur[cb], row, c * kWdBN + cb * 16 + g4, rn);
      }
      if (c + AHEAD < nch) load_x(c + AHEAD, xcur);   // lands during the following chunks' MFMAs
      __syncthreads();
    };
    if constexpr (AHEAD == 2) {
      for (int c = 0; c < nch; c += 2) {
        chunk(c, xc0);
        if (c + 1 < nch) chunk(c + 1, xc1);
      }
    } else {
      for (int c = 0; c < nch; ++c) chunk(c, xc0);
    }
    if (rownorm2) {
      if constexpr (VEC) {
        float t0 = rn, t1 = rn1;
        t0 += __shfl_xor(t0, 8);
        t1 += __shfl_xor(t1, 8);
        t0 += __shfl_xor(t0, 16);
        t1 += __shfl_xor(t1, 16);
        t0 += __shfl_xor(t0, 32);
        t1 += __shfl_xor(t1, 32);
        if (g4 == 0 && lo8) {
          if (rowA < M) rownorm2[rowA] = t0;
          if (rowB < M) rownorm2[rowB] = t1;
        }
      } else {
        float t = rn;
        t += __shfl_xor(t, 16);
        t += __shfl_xor(t, 32);
        if (g4 == 0 && row_ok) rownorm2[row] = t;
      }
    }
  }
}

// ------------------------------------------------------------------ TN split-K
constexpr int kTnBM = 64;

template <int NB, bool BF16>
__global__ __launch_bounds__(256) void gemm_tn_splitk_kernel(const float* __restrict__ A, int64_t R, int64_t M,
                                                             int64_t lda, const float* __restrict__ B, int64_t N,
                                                             int64_t ldb, float* __restrict__ partial,
                                                             int64_t chunk_rows, bool a_al, bool b_al, Gate gate) {
  if (gate_shut(gate)) return;
  constexpr int BN = NB * 16;
  constexpr int kTnBK = BF16 ? 32 : 16;   // rows per chunk: one MFMA K step
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
  float4 ra[kTnBK / 16], rb[B_SLOTS];
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < kTnBK / 16; ++q) {
      int r = (tid >> 4) + 16 * q, c4 = tid & 15;  // 16 rows x 16 float4 per slot
      int64_t row = k0 + r;
      ra[q] = row < r1 ? load4(A, lda, R, M, row, m0 + 4 * c4, a_al) : make_float4(0.f, 0.f, 0.f, 0.f);
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
#pragma unroll
    for (int q = 0; q < kTnBK / 16; ++q) {
      int r = (tid >> 4) + 16 * q, c4 = tid & 15;
      *reinterpret_cast<float4*>(&As[r * AW + 4 * c4]) = ra[q];
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
    // lane group g takes rows 4 g .. 4 g + 3 of each 16-row half of the chunk
    auto col4 = [&](const float* T, int w, int j, int h) {
      return make_float4(T[(16 * h + 4 * g + 0) * w + j], T[(16 * h + 4 * g + 1) * w + j],
                         T[(16 * h + 4 * g + 2) * w + j], T[(16 * h + 4 * g + 3) * w + j]);
    };
    if constexpr (BF16) {
      const s8v a = cat8(bf16x4(col4(As, AW, mi, 0)), bf16x4(col4(As, AW, mi, 1)));
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) {
        const int nj = cb * 16 + (lane & 15);
        acc[cb] = mfma_bf16_k32(a, cat8(bf16x4(col4(Bs, BW, nj, 0)), bf16x4(col4(Bs, BW, nj, 1))), acc[cb]);
      }
    } else {
      const float4 a = col4(As, AW, mi, 0);
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) mfma16_f32(a, col4(Bs, BW, cb * 16 + (lane & 15), 0), acc[cb]);
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
                                         int64_t ldg, Gate gate) {
  if (gate_shut(gate)) return;
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
                                                               int nblk, double* rsq, Gate gate) {
  if (gate_shut(gate)) return;
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

template <int NB, bool BF16>
int longk_reg_launch(hipStream_t st, const float* A, int64_t M, int64_t K, int64_t lda, const float* Bt, int64_t N,
                     int64_t ldb, float* C, int64_t ldc, int64_t nst, Gate gate) {
  const void* fn = (const void*)gemm_nt_longk_reg_kernel<NB, BF16>;
  constexpr int kLrThreads = lr_threads(BF16), kLrBM = 16 * (kLrThreads / 64);
  const int res = resident_blocks(fn, kLrThreads, 0);
  if (res <= 0) {
    set_error("gemm_nt_longk: no resident workgroup capacity reported");
    return SCS_EDEVICE;
  }
  const int64_t grid = std::min<int64_t>(cdiv(M, kLrBM), (int64_t)res);
  gemm_nt_longk_reg_kernel<NB, BF16><<<dim3((unsigned)grid), dim3(kLrThreads), 0, st>>>(A, M, K, lda, Bt, N, ldb, C,
                                                                                      ldc, nst, gate);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

template <bool BF16>
int longk_dispatch(hipStream_t st, int nb, const float* A, int64_t M, int64_t K, int64_t lda, const float* Bt,
                   int64_t N, int64_t ldb, float* C, int64_t ldc, int64_t nst, Gate gate) {
  if (aligned16(A, lda)) {
    switch (nb) {
      case 1: return longk_reg_launch<1, BF16>(st, A, M, K, lda, Bt, N, ldb, C, ldc, nst, gate);
      case 2: return longk_reg_launch<2, BF16>(st, A, M, K, lda, Bt, N, ldb, C, ldc, nst, gate);
      case 3: return longk_reg_launch<3, BF16>(st, A, M, K, lda, Bt, N, ldb, C, ldc, nst, gate);
      case 4: return longk_reg_launch<4, BF16>(st, A, M, K, lda, Bt, N, ldb, C, ldc, nst, gate);
      case 5: return longk_reg_launch<5, BF16>(st, A, M, K, lda, Bt, N, ldb, C, ldc, nst, gate);
      case 6: return longk_reg_launch<6, BF16>(st, A, M, K, lda, Bt, N, ldb, C, ldc, nst, gate);
      case 7: return longk_reg_launch<7, BF16>(st, A, M, K, lda, Bt, N, ldb, C, ldc, nst, gate);
      case 8: return longk_reg_launch<8, BF16>(st, A, M, K, lda, Bt, N, ldb, C, ldc, nst, gate);
      case 9: return longk_reg_launch<9, BF16>(st, A, M, K, lda, Bt, N, ldb, C, ldc, nst, gate);
      default: break;
    }
  }
  dim3 grid((unsigned)cdiv(M, kLkBM));
  bool aa = aligned16(A, lda), ba = aligned16(Bt, ldb);
#define SCS_LK(NBV) \
  case NBV:         \
    gemm_nt_longk_kernel<NBV, BF16><<<grid, 256, 0, st>>>(A, M, K, lda, Bt, N, ldb, C, ldc, nst, aa, ba, gate); break;
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
                int64_t ldb, float* partial, int64_t chunk_rows, int64_t nchunks, Gate gate) {
  if (aligned16(A, lda) && aligned16(B, ldb)) {
    const dim3 g((unsigned)cdiv(M, nb <= 4 ? tg_cols(4) : tg_cols(9)), (unsigned)nchunks), blk(kTgThreads);
#define SCS_TG(NBV)                                                                                        \
  case NBV:                                                                                                \
    gemm_tn_reg_kernel<NBV, BF16><<<g, blk, 0, st>>>(A, R, M, lda, B, N, ldb, partial, chunk_rows, gate); \
    break;
    switch (nb) {
      SCS_TG(1) SCS_TG(2) SCS_TG(3) SCS_TG(4) SCS_TG(5) SCS_TG(6) SCS_TG(7) SCS_TG(8) SCS_TG(9)
      default:
        set_error("gemm_tn_splitk: N > 144");
        return SCS_EINVAL;
    }
#undef SCS_TG
    SCS_HIP(hipGetLastError());
    return SCS_OK;
  }
  dim3 grid((unsigned)cdiv(M, kTnBM), (unsigned)nchunks);
  bool aa = aligned16(A, lda), ba = aligned16(B, ldb);
#define SCS_TN(NBV)                                                                                             \
  case NBV:                                                                                                     \
    gemm_tn_splitk_kernel<NBV, BF16><<<grid, 256, 0, st>>>(A, R, M, lda, B, N, ldb, partial, chunk_rows, aa, \
                                                           ba, gate);                                                 \
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
                         const float* Bt, int64_t N, int64_t ldb, float* C, int64_t ldc, bool pad16, Gate gate) {
  if (M <= 0 || N <= 0) return SCS_OK;
  int nb = (int)cdiv(N, 16);
  const int64_t nst = pad16 ? 16 * (int64_t)nb : N;   // columns N.. of the last 16 are zero
  if (nst > ldc) {
    set_error("gemm_nt_longk: ldc smaller than the stored width");
    return SCS_EINVAL;
  }
  return bf16 ? longk_dispatch<true>(st, nb, A, M, K, lda, Bt, N, ldb, C, ldc, nst, gate)
              : longk_dispatch<false>(st, nb, A, M, K, lda, Bt, N, ldb, C, ldc, nst, gate);
}

int gemm_wide_kpad(int64_t K) {
  const int64_t q = cdiv(K < 1 ? 1 : K, 16);
  return q <= 2 ? (int)(16 * q) : (q <= 4 ? 64 : (q <= 8 ? 128 : 160));
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
  const int KP = gemm_wide_kpad(K), NK = KP / 16;
  if (lda < KP || ldb < KP || !aligned16(A, lda) || !aligned16(Bt, ldb) || N > (1 << 30) ||
      cdiv(N, kWdBN) * kWdBN * ldb > (int64_t)1 << 31) {
    set_error("gemm_nt_wide: A and Bt need 16-byte aligned rows of at least gemm_wide_kpad(K) values, and Bt at "
              "most 2^31 elements (rows rounded up to 64)");
    return SCS_EINVAL;
  }
  const int Ni = (int)N, nq = (int)cdiv(K < 1 ? 1 : K, 16);
  const bool vec = N % 4 == 0 && (C0 == nullptr || aligned16(C0, ldc0)) &&
                   (out_bf16 ? ((uintptr_t)C % 8 == 0 && ldc % 4 == 0) : aligned16(C, ldc));
  const size_t bytes = bf16 ? (size_t)2 * kWdBN * (KP + 8) * 2 : (size_t)2 * kWdBN * (KP + 4) * 4;
  const void* fn = nullptr;
#define SCS_WD_PICK(NKV)                                                                                         \
  if (bf16) {                                                                                                    \
    if (out_bf16) fn = vec ? (const void*)gemm_nt_wide_kernel<true, true, NKV, true>                             \
                           : (const void*)gemm_nt_wide_kernel<true, true, NKV, false>;                           \
    else fn = vec ? (const void*)gemm_nt_wide_kernel<true, false, NKV, true>                                     \
                  : (const void*)gemm_nt_wide_kernel<true, false, NKV, false>;                                   \
  } else {                                                                                                       \
    if (out_bf16) fn = vec ? (const void*)gemm_nt_wide_kernel<false, true, NKV, true>                            \
                           : (const void*)gemm_nt_wide_kernel<false, true, NKV, false>;                          \
    else fn = vec ? (const void*)gemm_nt_wide_kernel<false, false, NKV, true>                                    \
                  : (const void*)gemm_nt_wide_kernel<false, false, NKV, false>;                                  \
  }
  switch (NK) {
    case 1: SCS_WD_PICK(1) break;
    case 2: SCS_WD_PICK(2) break;
    case 4: SCS_WD_PICK(4) break;
    case 8: SCS_WD_PICK(8) break;
    default: SCS_WD_PICK(10) break;
  }
#undef SCS_WD_PICK
  if (bytes > 65536) SCS_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  const int threads = wd_threads(NK);
  const int res = resident_blocks(fn, threads, bytes);
  if (res <= 0) {
    set_error("gemm_nt_wide: no resident workgroup capacity reported for this shape");
    return SCS_EDEVICE;
  }
  const int64_t grid = std::min<int64_t>(cdiv(M, 16 * (threads / 64)), (int64_t)res);
  void* args[] = {(void*)&A,    (void*)&M,    (void*)&lda,  (void*)&Bt,       (void*)&Ni,   (void*)&ldb,
                  (void*)&alpha, (void*)&C0,  (void*)&ldc0, (void*)&beta,     (void*)&beta_dev, (void*)&diag,
                  (void*)&diag_dev, (void*)&C, (void*)&ldc, (void*)&rownorm2, (void*)&nq};
  SCS_HIP(hipLaunchKernel(fn, dim3((unsigned)grid), dim3(threads), args, bytes, st));
  return SCS_OK;
}

int64_t gemm_tn_splitk_chunks(int64_t R, int64_t M, int64_t N, const float* A, int64_t lda, const float* B,
                              int64_t ldb) {
  if (R <= 0 || M <= 0 || N <= 0) return 1;
  if (aligned16(A, lda) && aligned16(B, ldb)) {
    // one workgroup per CU is resident: as many row chunks as fill the device once
    const int nb = (int)cdiv(N, 16);
    const int64_t slabs = cdiv(M, nb <= 4 ? tg_cols(4) : tg_cols(9));
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                 hipSuccess)
      cus = 256;
    return std::max<int64_t>(1, std::min<int64_t>(cdiv(R, 256), cus / slabs));
  }
  return std::max<int64_t>(1, std::min<int64_t>(cdiv(R, 512), std::max<int64_t>(1, 1024 / cdiv(M, 64))));
}

int launch_gemm_tn_splitk(hipStream_t st, int bf16, const float* A, int64_t R, int64_t M, int64_t lda,
                          const float* B, int64_t N, int64_t ldb, float* partial, int64_t chunk_rows,
                          int64_t nchunks, Gate gate) {
  if (M <= 0 || N <= 0) return SCS_OK;
  int nb = (int)cdiv(N, 16);
  return bf16 ? tn_dispatch<true>(st, nb, A, R, M, lda, B, N, ldb, partial, chunk_rows, nchunks, gate)
              : tn_dispatch<false>(st, nb, A, R, M, lda, B, N, ldb, partial, chunk_rows, nchunks, gate);
}

int launch_reduce_partials_t(hipStream_t st, const float* partial, int64_t nchunks, int64_t d, int Pc, double* G,
                             int64_t ldg, Gate gate) {
  if (d * Pc <= 0) return SCS_OK;
  reduce_partials_t_kernel<<<dim3((unsigned)cdiv(d * Pc, 256)), dim3(256), 0, st>>>(partial, nchunks, d, Pc, G, ldg, gate);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_residual_batched(hipStream_t st, float* R, int64_t n, int P, const float* Y, int ny, int nblk,
                            double* rsq, Gate gate) {
  if (n <= 0 || P <= 0) return SCS_OK;
  residual_batched_kernel<<<dim3((unsigned)nblk), dim3(256), 0, st>>>(R, n, P, Y, ny, nblk, rsq, gate);
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

// rows per workgroup: a multiple of the slab, for about min(256, R / 512) workgroups
static int64_t gram_rr_f32_chunk(int64_t R) {
  const int64_t target = std::max<int64_t>(1, std::min<int64_t>(256, cdiv(R, 512)));
  return cdiv(cdiv(R, target), (int64_t)kGramSlab) * kGramSlab;
}

int64_t gram_rr_f32_parts(int64_t R) { return R <= 0 ? 1 : cdiv(R, gram_rr_f32_chunk(R)); }

int launch_gram_rr_f32(hipStream_t st, const float* W, int64_t R, int L, int64_t ldw, float* partial) {
  if (R <= 0 || L <= 0) return SCS_OK;
  if (L > 64 || ldw < L) return SCS_EINVAL;
  const int64_t chunk = gram_rr_f32_chunk(R);
  gram_rr_f32_kernel<<<(unsigned)cdiv(R, chunk), 256, 0, st>>>(W, R, L, ldw, chunk, partial);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

}  // namespace scs
