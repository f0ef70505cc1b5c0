// SVRG inner loop (Alg. 1, the m steps of one epoch) as one persistent launch.
//
// The iterate is kept as the correction delta = w_t - w~ (w~ the snapshot): each step
//   c_j   = a_{i_j}^T delta                         (b dot products, i_j drawn from q)
//   delta = delta - eta ((1/b) sum_j c_j a_{i_j} / (n q_{i_j}) + mu)
//   sum  += delta                                   (for the averaged snapshot)
// which is the variance-reduced step of Alg. 1 for the components 1/2 (n+d)/n (a_i^T w - t_i)^2:
// grad f_i(w_{t-1}) - grad f_i(w~) = (n+d)/n (a_i^T delta) a_i, divided by (n+d) q_i.
// Working on delta keeps FP32 rounding relative to the shrinking correction.
//
// Columns are split over W cooperating workgroups (each on its own CU); a workgroup holds its
// slice of delta, mu and sum in registers (replicated over its 8 row groups) and gathers only
// its slice of the b rows. The b partial dot products of a step are exchanged through global
// memory: every workgroup posts its partials and a step counter, then sums all W partials in
// the same fixed order, so all workgroups compute bit-identical c_j. Waits are bounded: a wait
// that exceeds its poll budget raises an abort flag that ends every workgroup's loop.
// Rows of the next step are loaded while the current step's reductions run (the index stream
// does not depend on the iterate).
#include "scs_internal.h"

namespace scs {



namespace {

constexpr int kInnerThreads = 256;
constexpr uint32_t kPollBudget = 1u << 22;
constexpr int kMaxPairs = 4;  // exchange words gathered per thread: W * b <= 4 * 256

// Barrier for LDS traffic only: waits for this wave's LDS operations but not for its
// outstanding global loads (the prefetched rows of the next step stay in flight).
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

template <bool BF16>
__device__ __forceinline__ float4 row_load(const void* base, int64_t ld, int64_t row, int64_t col, int64_t d) {
  if constexpr (BF16) {
    const uint16_t* p = reinterpret_cast<const uint16_t*>(base) + row * ld + col;
    if (col + 3 < d) {
      uint2 u = *reinterpret_cast<const uint2*>(p);
      return make_float4(__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xffff0000u),
                         __uint_as_float(u.y << 16), __uint_as_float(u.y & 0xffff0000u));
    }
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (col + 0 < d) v.x = bf16_to_f32(p[0]);
    if (col + 1 < d) v.y = bf16_to_f32(p[1]);
    if (col + 2 < d) v.z = bf16_to_f32(p[2]);
    return v;
  } else {
    const float* p = reinterpret_cast<const float*>(base) + row * ld + col;
    if (col + 3 < d) return *reinterpret_cast<const float4*>(p);
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (col + 0 < d) v.x = p[0];
    if (col + 1 < d) v.y = p[1];
    if (col + 2 < d) v.z = p[2];
    return v;
  }
}

__device__ __forceinline__ float f4get(const float4& v, int i) { return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w; }

template <int RPT, int CPT, bool BF16>
__global__ __launch_bounds__(kInnerThreads) void inner_epoch_kernel(InnerArgs a) {
  const int bid = blockIdx.x;
  if (bid % a.xcd_stride != 0) return;
  const int w = bid / a.xcd_stride;
  if (w >= a.W) return;
  if (a.state->done) return;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int cgt = lane & 31;
  const int rg = wave * 2 + (lane >> 5);
  const int b = a.b, W = a.W;
  const int64_t NR = a.n + a.d;
  const int64_t c_begin = (int64_t)w * a.slice;
  const int64_t c_end = c_begin + a.slice < a.d ? c_begin + a.slice : a.d;
  uint64_t* xb = a.xbuf;

  __shared__ float pd[64][33];
  __shared__ float gam[64];
  __shared__ float xs[16][64];
  __shared__ float4 red[8][32 * CPT];
  __shared__ int s_abort;

  float dl[CPT][4], sm[CPT][4], smc[CPT][4], muv[CPT][4], w0[CPT][4];
  int64_t col[CPT];
#pragma unroll
  for (int q = 0; q < CPT; ++q) {
    col[q] = c_begin + 4 * (cgt + 32 * q);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      int64_t c = col[q] + v;
      bool ok = c < c_end;
      muv[q][v] = ok ? a.mu[c] : 0.f;
      w0[q][v] = ok ? a.wt[c] : 0.f;
      dl[q][v] = 0.f;
      sm[q][v] = 0.f;
      smc[q][v] = 0.f;
    }
  }
  const float eta = a.eta_from_state ? (float)(a.step_scale * (double)a.n / a.state->beta_sum) : (float)a.eta;
  if (tid == 0) s_abort = 0;

  // component indices of this thread's rows for a step (0 for rows j >= b)
  auto load_idx = [&](int64_t t, int32_t (&ix)[RPT]) {
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      int j = rg + 8 * q;
      int32_t i = (j < b && t < a.m) ? a.idx[t * b + j] : 0;
      ix[q] = ((uint64_t)(int64_t)i >= (uint64_t)NR) ? 0 : i;  // out-of-range injected index: stay in bounds
    }
  };
  auto load_rows = [&](const int32_t (&ix)[RPT], float4 (&buf)[RPT][CPT]) {
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      int j = rg + 8 * q;
      int64_t i = ix[q];
      const void* base = i < a.n ? a.Xt : a.reg;
      int64_t ld = i < a.n ? a.ldx : a.ldr;
      int64_t row = i < a.n ? i : i - a.n;
#pragma unroll
      for (int c = 0; c < CPT; ++c)
        buf[q][c] = (j < b && col[c] < c_end) ? row_load<BF16>(base, ld, row, col[c], c_end)
                                              : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };

  float4 cur[RPT][CPT], nxt[RPT][CPT];
  int32_t ix_next[RPT];
  {
    int32_t ix0[RPT];
    load_idx(0, ix0);
    load_rows(ix0, cur);
    load_idx(1, ix_next);
  }
  float sc_cur = (tid < b) ? a.scale[tid] : 0.f;
  lds_barrier();
  for (int64_t t = 0; t < a.m; ++t) {
    // prefetch: rows of step t+1 (indices loaded one step ago), indices of step t+2
    if (t + 1 < a.m) load_rows(ix_next, nxt);
    load_idx(t + 2, ix_next);
    const float sc_next = (tid < b && t + 1 < a.m) ? a.scale[(t + 1) * b + tid] : 0.f;
    // partial dot products over this workgroup's columns
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      float p = 0.f;
#pragma unroll
      for (int c = 0; c < CPT; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) p = fmaf(f4get(cur[q][c], v), dl[c][v], p);
      int j = rg + 8 * q;
      if (j < b) pd[j][cgt] = p;
    }
    lds_barrier();
    float cl = 0.f;
    if (tid < b) {
#pragma unroll 8
      for (int g = 0; g < 32; ++g) cl += pd[tid][g];
    }
    if (W > 1) {
      // post (value, step tag) as one 64-bit word, then gather all W x b words in parallel;
      // a word is valid once its tag equals this step's, so no fence is needed
      const int par = (int)(t & 1);
      const uint32_t target = a.step_base + (uint32_t)t + 1u;
      uint64_t* slot = xb + (int64_t)par * W * 64;
      if (tid < b)
        __hip_atomic_store(&slot[(int64_t)w * 64 + tid], ((uint64_t)target << 32) | __float_as_uint(cl),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      uint64_t xv[kMaxPairs];
      bool need[kMaxPairs];
#pragma unroll
      for (int q = 0; q < kMaxPairs; ++q) {
        int pidx = tid + kInnerThreads * q;
        need[q] = pidx < W * b;
        xv[q] = 0;
        if (need[q]) {
          int v = pidx / b, j = pidx - v * b;
          xv[q] = __hip_atomic_load(&slot[(int64_t)v * 64 + j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      uint32_t polls = 0;
      bool bad = false;
      for (;;) {
        bool pending = false;
#pragma unroll
        for (int q = 0; q < kMaxPairs; ++q) pending |= need[q] && (uint32_t)(xv[q] >> 32) != target;
        if (!pending) break;
        if (++polls > kPollBudget ||
            __hip_atomic_load(&a.state->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == SCS_EDEVICE) {
          bad = true;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
#pragma unroll
        for (int q = 0; q < kMaxPairs; ++q) {
          if (need[q] && (uint32_t)(xv[q] >> 32) != target) {
            int pidx = tid + kInnerThreads * q;
            int v = pidx / b, j = pidx - v * b;
            xv[q] = __hip_atomic_load(&slot[(int64_t)v * 64 + j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
        }
      }
      if (bad) {
        s_abort = 1;
        __hip_atomic_store(&a.state->status, SCS_EDEVICE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&a.state->done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
#pragma unroll
      for (int q = 0; q < kMaxPairs; ++q) {
        if (need[q]) {
          int pidx = tid + kInnerThreads * q;
          int v = pidx / b, j = pidx - v * b;
          xs[v][j] = __uint_as_float((uint32_t)xv[q]);
        }
      }
      lds_barrier();
      if (tid < b) {
        float s = 0.f;
        for (int v = 0; v < W; ++v) s += xs[v][tid];  // same order in every workgroup
        cl = s;
      }
    }
    if (tid < b) gam[tid] = sc_cur * cl / (float)b;
    lds_barrier();
    if (s_abort) break;
    // (1/b) sum_j c_j a_j / (n q_j) over this thread's rows, then across the 8 row groups
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      float u[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        int j = rg + 8 * q;
        float gj = j < b ? gam[j] : 0.f;
#pragma unroll
        for (int v = 0; v < 4; ++v) u[v] = fmaf(gj, f4get(cur[q][c], v), u[v]);
      }
      red[rg][cgt + 32 * c] = make_float4(u[0], u[1], u[2], u[3]);
    }
    lds_barrier();
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      float tot[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int g = 0; g < 8; ++g) {
        float4 r = red[g][cgt + 32 * c];
        tot[0] += r.x;
        tot[1] += r.y;
        tot[2] += r.z;
        tot[3] += r.w;
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        dl[c][v] -= eta * (tot[v] + muv[c][v]);
        float y = dl[c][v] - smc[c][v];
        float s2 = sm[c][v] + y;
        smc[c][v] = (s2 - sm[c][v]) - y;
        sm[c][v] = s2;
      }
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q)
#pragma unroll
      for (int c = 0; c < CPT; ++c) cur[q][c] = nxt[q][c];
    sc_cur = sc_next;
  }

  if (!s_abort && rg == 0) {
    const float inv_m = 1.0f / (float)a.m;
#pragma unroll
    for (int q = 0; q < CPT; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int64_t c = col[q] + v;
        if (c < c_end) {
          if (a.wt_prev) a.wt_prev[c] = w0[q][v];
          float upd = a.average ? (sm[q][v] - smc[q][v]) * inv_m : dl[q][v];
          a.wt[c] = w0[q][v] + upd;
        }
      }
  }
  if (w == 0 && tid == 0 && !s_abort) {
    a.state->epochs += 1;
    a.state->eta = (double)eta;
  }
}

template <int RPT, int CPT, bool BF16>
int launch_t(hipStream_t st, InnerArgs& a) {
  dim3 grid((unsigned)(a.W * a.xcd_stride)), block(kInnerThreads);
  if (a.W > 1) {
    void* args[] = {&a};
    SCS_HIP(hipLaunchCooperativeKernel((const void*)inner_epoch_kernel<RPT, CPT, BF16>, grid, block, args, 0, st));
  } else {
    inner_epoch_kernel<RPT, CPT, BF16><<<grid, block, 0, st>>>(a);
    SCS_HIP(hipGetLastError());
  }
  return SCS_OK;
}

template <int RPT, bool BF16>
int launch_c(hipStream_t st, InnerArgs& a, int cpt) {
  switch (cpt) {
    case 1: return launch_t<RPT, 1, BF16>(st, a);
    case 2: return launch_t<RPT, 2, BF16>(st, a);
    case 3: return launch_t<RPT, 3, BF16>(st, a);
    case 4: return launch_t<RPT, 4, BF16>(st, a);
  }
  set_error("inner loop: column slice too wide (more than 512 columns per workgroup)");
  return SCS_EINVAL;
}

}  // namespace

int inner_default_workgroups(int64_t d) {
  int64_t W = cdiv(d, 128);
  if (W < 1) W = 1;
  if (W > 16) W = 16;
  return (int)W;
}

int launch_inner_epoch(hipStream_t st, InnerArgs& a, int bf16) {
  if (a.b < 1 || a.b > 64 || a.m < 1 || a.W < 1 || a.W > 16) {
    set_error("inner loop: need 1 <= b <= 64, m >= 1, 1 <= workgroups <= 16");
    return SCS_EINVAL;
  }
  if (a.ldx % 4 != 0 || a.ldr % 4 != 0) {
    set_error("inner loop: row strides must be multiples of 4 elements");
    return SCS_EINVAL;
  }
  a.slice = cdiv(cdiv(a.d, a.W), 4) * 4;
  int cpt = (int)cdiv(a.slice, 128);
  int rpt = (int)cdiv(a.b, 8);
  if (rpt <= 1) return bf16 ? launch_c<1, true>(st, a, cpt) : launch_c<1, false>(st, a, cpt);
  if (rpt <= 2) return bf16 ? launch_c<2, true>(st, a, cpt) : launch_c<2, false>(st, a, cpt);
  if (rpt <= 4) return bf16 ? launch_c<4, true>(st, a, cpt) : launch_c<4, false>(st, a, cpt);
  return bf16 ? launch_c<8, true>(st, a, cpt) : launch_c<8, false>(st, a, cpt);
}

}  // namespace scs
