// Full-gradient pass of SVRG (Alg. 1, the gradient at the snapshot), streamed from HBM once:
//   r_i = x_i^T w - y_i,   g_partial = sum_i r_i x_i,   rsq_partial = sum_i r_i^2
// over a contiguous block of rows per workgroup. Each row is read once into registers, used
// for its dot product and then for the accumulation (the two GEMV halves are fused).
// One wave owns one row at a time; lane l holds columns (c*64 + l)*VEC + v, so the per-lane
// gradient accumulator covers the same columns for every row. Accumulation is compensated
// (Kahan) in FP32; workgroup partials are summed in FP64 by grad_finish.
#include "scs_internal.h"

namespace scs {

namespace {

constexpr int kGradThreads = 256;
constexpr int kGradWaves = kGradThreads / 64;

template <int VEC>
struct VecT;
template <>
struct VecT<4> {
  using T = float4;
};
template <>
struct VecT<1> {
  using T = float;
};

// X is streamed once per pass: non-temporal loads keep it from displacing reused data in the caches
typedef float f4v_nt __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void vload(const float* p, float4& v) {
  const f4v_nt t = __builtin_nontemporal_load(reinterpret_cast<const f4v_nt*>(p));
  v = make_float4(t.x, t.y, t.z, t.w);
}
__device__ __forceinline__ void vload(const float* p, float& v) { v = __builtin_nontemporal_load(p); }
__device__ __forceinline__ float comp(const float4& v, int i) { return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w; }
__device__ __forceinline__ float comp(const float& v, int) { return v; }

// Workgroup wg of nwg covering rows [wg ceil(n/nwg), (wg+1) ceil(n/nwg)) of one problem.
template <int VEC, int NCH>
__device__ __forceinline__ void grad_partial_body(const float* __restrict__ X, int64_t n, int64_t d, int64_t ldx,
                                                  const float* __restrict__ y, const float* __restrict__ w,
                                                  float* __restrict__ part, double* __restrict__ rsq_part,
                                                  int64_t wg, int64_t nwg) {
  using V = typename VecT<VEC>::T;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t rows_per_wg = cdiv(n, nwg);
  const int64_t r0 = wg * rows_per_wg;
  const int64_t r1 = r0 + rows_per_wg < n ? r0 + rows_per_wg : n;

  float wv[NCH][VEC], acc[NCH][VEC], cmp[NCH][VEC];
  bool valid[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    int64_t col = (int64_t)(c * 64 + lane) * VEC;
    valid[c] = col < d;
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      wv[c][v] = valid[c] ? w[col + v] : 0.f;
      acc[c][v] = 0.f;
      cmp[c][v] = 0.f;
    }
  }
  double rsq = 0.0;

  // Rows are taken in pairs (r, r + 4) per wave, and the next pair's loads are issued before the
  // current pair is reduced (two pairs in flight per wave). Prefetch addresses past the block are
  // clamped to row n - 1 and never used.
  int64_t r = r0 + wave;
  constexpr int64_t kStep = 2 * kGradWaves;
  auto load_pair = [&](int64_t rr, V (&A)[NCH], V (&Bv)[NCH], float& ya_, float& yb_) {
    const int64_t ra = rr < n ? rr : n - 1;
    const int64_t rb = rr + kGradWaves < n ? rr + kGradWaves : n - 1;
    const float* pa = X + ra * ldx;
    const float* pb = X + rb * ldx;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      int64_t col = (int64_t)(c * 64 + lane) * VEC;
      if (valid[c]) {
        vload(pa + col, A[c]);
        vload(pb + col, Bv[c]);
      } else {
        A[c] = V{};
        Bv[c] = V{};
      }
    }
    ya_ = y[ra];
    yb_ = y[rb];
  };
  auto reduce_pair = [&](const V (&xa)[NCH], const V (&xb)[NCH], float ya, float yb) {
    float da = 0.f, db = 0.f;
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        da = fmaf(comp(xa[c], v), wv[c][v], da);
        db = fmaf(comp(xb[c], v), wv[c][v], db);
      }
    da = warp_sum(da) - ya;
    db = warp_sum(db) - yb;
    rsq += (double)da * da + (double)db * db;
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        // Kahan: acc += da*xa + db*xb with the rounding error carried in cmp
        float t1 = fmaf(da, comp(xa[c], v), -cmp[c][v]);
        float s1 = acc[c][v] + t1;
        cmp[c][v] = (s1 - acc[c][v]) - t1;
        acc[c][v] = s1;
        float t2 = fmaf(db, comp(xb[c], v), -cmp[c][v]);
        float s2 = acc[c][v] + t2;
        cmp[c][v] = (s2 - acc[c][v]) - t2;
        acc[c][v] = s2;
      }
  };
  if (r + kGradWaves < r1) {
    V xa[NCH], xb[NCH], na[NCH], nb[NCH];
    float ya, yb, nya, nyb;
    load_pair(r, xa, xb, ya, yb);
    for (;;) {
      load_pair(r + kStep, na, nb, nya, nyb);
      reduce_pair(xa, xb, ya, yb);
      r += kStep;
      if (!(r + kGradWaves < r1)) break;
      load_pair(r + kStep, xa, xb, ya, yb);
      reduce_pair(na, nb, nya, nyb);
      r += kStep;
      if (!(r + kGradWaves < r1)) break;
    }
  }
  for (; r < r1; r += kGradWaves) {
    V xa[NCH];
    const float* pa = X + r * ldx;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      int64_t col = (int64_t)(c * 64 + lane) * VEC;
      if (valid[c]) vload(pa + col, xa[c]);
      else xa[c] = V{};
    }
    float da = 0.f;
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
      for (int v = 0; v < VEC; ++v) da = fmaf(comp(xa[c], v), wv[c][v], da);
    da = warp_sum(da) - y[r];
    rsq += (double)da * da;
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        float t1 = fmaf(da, comp(xa[c], v), -cmp[c][v]);
        float s1 = acc[c][v] + t1;
        cmp[c][v] = (s1 - acc[c][v]) - t1;
        acc[c][v] = s1;
      }
  }

  // combine the waves of the workgroup through LDS (fixed order: wave 0 + 1 + 2 + 3)
  __shared__ float sbuf[kGradWaves - 1][NCH * 64 * VEC];
  __shared__ double srsq[kGradWaves];
  if (lane == 0) srsq[wave] = rsq;
  if (wave > 0) {
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
      for (int v = 0; v < VEC; ++v) sbuf[wave - 1][(c * 64 + lane) * VEC + v] = acc[c][v] - cmp[c][v];
  }
  __syncthreads();
  if (wave == 0) {
    float* out = part + wg * d;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      int64_t col = (int64_t)(c * 64 + lane) * VEC;
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        float s = acc[c][v] - cmp[c][v];
        for (int q = 0; q < kGradWaves - 1; ++q) s += sbuf[q][(c * 64 + lane) * VEC + v];
        if (valid[c] && col + v < d) out[col + v] = s;
      }
    }
    if (lane == 0) {
      double t = 0.0;
      for (int q = 0; q < kGradWaves; ++q) t += srsq[q];
      rsq_part[wg] = t;
    }
  }
}

// Column-split variant for rows too wide to sit in one wave's registers (d > 2048, 16-byte aligned
// rows). The four waves of a workgroup share every row: wave q holds columns [256 NCW q, 256 NCW (q + 1))
// (lane l, chunk c: columns 256 NCW q + 4 (64 c + l) .. + 3). For each row pair the waves' partial dot
// products meet in LDS (two slots, one barrier per pair) and are added in wave order 0, 1, 2, 3, so all
// waves hold the same r_i; each wave then accumulates r_i x_i over its own columns (Kahan), and wave 0
// alone adds r_i^2. The next pair's loads are issued before the current pair is reduced.
template <int NCW>
__device__ __forceinline__ void grad_partial_split_body(const float* __restrict__ X, int64_t n, int64_t d,
                                                        int64_t ldx, const float* __restrict__ y,
                                                        const float* __restrict__ w, float* __restrict__ part,
                                                        double* __restrict__ rsq_part, int64_t wg, int64_t nwg) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t rows_per_wg = cdiv(n, nwg);
  const int64_t r0 = wg * rows_per_wg;
  const int64_t r1 = r0 + rows_per_wg < n ? r0 + rows_per_wg : n;
  const int64_t cbase = (int64_t)wave * 256 * NCW;

  float4 wv[NCW];
  float acc[NCW][4], cmp[NCW][4];
  bool valid[NCW];
#pragma unroll
  for (int c = 0; c < NCW; ++c) {
    const int64_t col = cbase + 4 * (c * 64 + lane);
    valid[c] = col < d;   // d % 4 == 0: a quad is wholly inside or outside
    wv[c] = valid[c] ? make_float4(w[col], w[col + 1], w[col + 2], w[col + 3]) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[c][v] = cmp[c][v] = 0.f;
  }
  double rsq = 0.0;
  __shared__ float sdot[2][kGradWaves][2];
  int slot = 0;

  auto load_pair = [&](int64_t rr, float4 (&A)[NCW], float4 (&B)[NCW], float& ya_, float& yb_) {
    const int64_t ra = rr, rb = rr + 1 < r1 ? rr + 1 : rr;
#pragma unroll
    for (int c = 0; c < NCW; ++c) {
      const int64_t col = cbase + 4 * (c * 64 + lane);
      if (valid[c]) {
        vload(X + ra * ldx + col, A[c]);
        vload(X + rb * ldx + col, B[c]);
      } else {
        A[c] = B[c] = make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
    ya_ = y[ra];
    yb_ = y[rb];
  };
  auto kahan = [&](float r, const float4 (&A)[NCW]) {
#pragma unroll
    for (int c = 0; c < NCW; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float t = fmaf(r, comp(A[c], v), -cmp[c][v]);
        const float s1 = acc[c][v] + t;
        cmp[c][v] = (s1 - acc[c][v]) - t;
        acc[c][v] = s1;
      }
  };
  // rows rr and rr + 1 (has_b false: the pair is the block's last row alone)
  auto reduce_pair = [&](const float4 (&A)[NCW], const float4 (&B)[NCW], float ya, float yb, bool has_b) {
    float da = 0.f, db = 0.f;
#pragma unroll
    for (int c = 0; c < NCW; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        da = fmaf(comp(A[c], v), comp(wv[c], v), da);
        db = fmaf(comp(B[c], v), comp(wv[c], v), db);
      }
    da = warp_sum(da);
    db = warp_sum(db);
    if (lane == 0) {
      sdot[slot][wave][0] = da;
      sdot[slot][wave][1] = db;
    }
    __syncthreads();
    float sa = sdot[slot][0][0], sb = sdot[slot][0][1];
#pragma unroll
    for (int q = 1; q < kGradWaves; ++q) {
      sa += sdot[slot][q][0];
      sb += sdot[slot][q][1];
    }
    slot ^= 1;   // the other slot was last read before this pair's barrier
    sa -= ya;
    sb -= yb;
    if (wave == 0) rsq += (double)sa * sa + (has_b ? (double)sb * sb : 0.0);
    kahan(sa, A);
    if (has_b) kahan(sb, B);
  };

  if (r0 < r1) {
    float4 xa[NCW], xb[NCW], na[NCW], nb[NCW];
    float ya, yb, nya, nyb;
    int64_t r = r0;   // uniform over the workgroup, so every barrier is reached by all waves
    load_pair(r, xa, xb, ya, yb);
    for (;;) {
      const bool more = r + 2 < r1;
      if (more) load_pair(r + 2, na, nb, nya, nyb);
      reduce_pair(xa, xb, ya, yb, r + 1 < r1);
      r += 2;
      if (!more) break;
      const bool more2 = r + 2 < r1;
      if (more2) load_pair(r + 2, xa, xb, ya, yb);
      reduce_pair(na, nb, nya, nyb, r + 1 < r1);
      r += 2;
      if (!more2) break;
    }
  }

  float* out = part + wg * d;
#pragma unroll
  for (int c = 0; c < NCW; ++c) {
    const int64_t col = cbase + 4 * (c * 64 + lane);
    if (valid[c]) {
#pragma unroll
      for (int v = 0; v < 4; ++v) out[col + v] = acc[c][v] - cmp[c][v];
    }
  }
  if (wave == 0 && lane == 0) rsq_part[wg] = rsq;
}

template <int NCW>
__global__ __launch_bounds__(kGradThreads) void grad_partial_split_kernel(const float* __restrict__ X, int64_t n,
                                                                          int64_t d, int64_t ldx,
                                                                          const float* __restrict__ y,
                                                                          const float* __restrict__ w,
                                                                          float* __restrict__ part,
                                                                          double* __restrict__ rsq_part,
                                                                          const SolveState* state) {
  if (state && state->done) return;
  grad_partial_split_body<NCW>(X, n, d, ldx, y, w, part, rsq_part, blockIdx.x, gridDim.x);
}

template <int VEC, int NCH>
__global__ __launch_bounds__(kGradThreads) void grad_partial_kernel(const float* __restrict__ X, int64_t n,
                                                                    int64_t d, int64_t ldx,
                                                                    const float* __restrict__ y,
                                                                    const float* __restrict__ w,
                                                                    float* __restrict__ part,
                                                                    double* __restrict__ rsq_part,
                                                                    const SolveState* state) {
  if (state && state->done) return;
  grad_partial_body<VEC, NCH>(X, n, d, ldx, y, w, part, rsq_part, blockIdx.x, gridDim.x);
}

// All problems of a batch in one launch: problem p owns workgroups [wg_prefix[p], wg_prefix[p+1]).
// Workgroups [base, base + gridDim.x) of the batch's flattened grid (problems sharing one row layout
// are launched together).
template <int VEC, int NCH>
__global__ __launch_bounds__(kGradThreads) void grad_partial_batched_kernel(const BatchProb* P, int nprob,
                                                                            const int64_t* wg_prefix, int64_t base) {
  const int64_t x = base + blockIdx.x;
  const int p = find_prob(wg_prefix, nprob, x);
  const BatchProb& q = P[p];
  if (q.state->done) return;
  grad_partial_body<VEC, NCH>(q.X, q.n, q.d, q.ldx, q.y, q.w32, q.gpart, q.grsq, x - wg_prefix[p], q.nwg);
}

template <int VEC, int NCH>
int launch_t(hipStream_t st, const float* X, int64_t n, int64_t d, int64_t ldx, const float* y, const float* w,
             float* part, double* rsq_part, int nwg, const SolveState* state) {
  grad_partial_kernel<VEC, NCH><<<nwg, kGradThreads, 0, st>>>(X, n, d, ldx, y, w, part, rsq_part, state);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

template <int NCW>
int launch_split(hipStream_t st, const float* X, int64_t n, int64_t d, int64_t ldx, const float* y, const float* w,
                 float* part, double* rsq_part, int nwg, const SolveState* state) {
  grad_partial_split_kernel<NCW><<<nwg, kGradThreads, 0, st>>>(X, n, d, ldx, y, w, part, rsq_part, state);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

template <int VEC, int NCH>
int launch_bt(hipStream_t st, const BatchProb* P, int nprob, const int64_t* wg_prefix, int64_t base, int64_t count) {
  grad_partial_batched_kernel<VEC, NCH><<<(unsigned)count, kGradThreads, 0, st>>>(P, nprob, wg_prefix, base);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

}  // namespace

int launch_grad_partial_batched(hipStream_t st, const BatchProb* P, int nprob, const int64_t* wg_prefix,
                                int64_t base, int64_t count, int64_t max_d, int vec4) {
  if (nprob < 1 || count < 1) return SCS_OK;
  if (vec4) {
    int64_t nch = cdiv(max_d, 256);
    if (nch <= 1) return launch_bt<4, 1>(st, P, nprob, wg_prefix, base, count);
    if (nch <= 2) return launch_bt<4, 2>(st, P, nprob, wg_prefix, base, count);
    if (nch <= 4) return launch_bt<4, 4>(st, P, nprob, wg_prefix, base, count);
    if (nch <= 8) return launch_bt<4, 8>(st, P, nprob, wg_prefix, base, count);
  } else {
    int64_t nch = cdiv(max_d, 64);
    if (nch <= 1) return launch_bt<1, 1>(st, P, nprob, wg_prefix, base, count);
    if (nch <= 2) return launch_bt<1, 2>(st, P, nprob, wg_prefix, base, count);
    if (nch <= 4) return launch_bt<1, 4>(st, P, nprob, wg_prefix, base, count);
    if (nch <= 8) return launch_bt<1, 8>(st, P, nprob, wg_prefix, base, count);
    if (nch <= 16) return launch_bt<1, 16>(st, P, nprob, wg_prefix, base, count);
  }
  set_error("batched full gradient: d too large for the register-resident row layout");
  return SCS_EINVAL;
}

int grad_num_workgroups(int64_t n, int64_t d) {
  (void)d;
  int64_t want = 512;  // 2 per CU on 256 CUs (measured: 1024 and 2048 are slower, more rows per wave pipeline better)
  int64_t by_rows = cdiv(n, 8);
  return (int)(want < by_rows ? want : (by_rows < 1 ? 1 : by_rows));
}

int launch_grad_partial(hipStream_t st, const float* X, int64_t n, int64_t d, int64_t ldx, const float* y,
                        const float* w, float* part, double* rsq_part, int nwg, const SolveState* state) {
  bool vec4 = (d % 4 == 0) && (ldx % 4 == 0) && ((uintptr_t)X % 16 == 0);
  if (vec4) {
    int64_t nch = cdiv(d, 256);
    if (nch <= 1) return launch_t<4, 1>(st, X, n, d, ldx, y, w, part, rsq_part, nwg, state);
    if (nch <= 2) return launch_t<4, 2>(st, X, n, d, ldx, y, w, part, rsq_part, nwg, state);
    if (nch <= 4) return launch_t<4, 4>(st, X, n, d, ldx, y, w, part, rsq_part, nwg, state);
    if (nch <= 8) return launch_t<4, 8>(st, X, n, d, ldx, y, w, part, rsq_part, nwg, state);
    // wider rows: columns split over the workgroup's waves (a row per wave spilled registers at d = 5000)
    if (nch <= 12) return launch_split<3>(st, X, n, d, ldx, y, w, part, rsq_part, nwg, state);
    if (nch <= 16) return launch_split<4>(st, X, n, d, ldx, y, w, part, rsq_part, nwg, state);
    if (nch <= 20) return launch_split<5>(st, X, n, d, ldx, y, w, part, rsq_part, nwg, state);
    if (nch <= 32) return launch_split<8>(st, X, n, d, ldx, y, w, part, rsq_part, nwg, state);
  } else {
    int64_t nch = cdiv(d, 64);
    if (nch <= 1) return launch_t<1, 1>(st, X, n, d, ldx, y, w, part, rsq_part, nwg, state);
    if (nch <= 2) return launch_t<1, 2>(st, X, n, d, ldx, y, w, part, rsq_part, nwg, state);
    if (nch <= 4) return launch_t<1, 4>(st, X, n, d, ldx, y, w, part, rsq_part, nwg, state);
    if (nch <= 8) return launch_t<1, 8>(st, X, n, d, ldx, y, w, part, rsq_part, nwg, state);
    if (nch <= 16) return launch_t<1, 16>(st, X, n, d, ldx, y, w, part, rsq_part, nwg, state);
  }
  set_error("full gradient: d too large for the register-resident row layout");
  return SCS_EINVAL;
}

}  // namespace scs
