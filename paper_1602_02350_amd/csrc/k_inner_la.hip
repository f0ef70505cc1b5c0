// SVRG inner loop (Alg. 1, the m steps of one epoch) with the next step's dot products prepared while
// the current step's exchange is in flight.
//
// The persistent kernel of k_inner.hip spends each step in a chain: the cross-workgroup exchange of the
// b partial dot products c_t = R_t delta_t, then the update delta_{t+1} = delta_t - eta (R_t^T g_t + mu)
// (g_t = the step's coefficients scale_j c_j / b), then the next dot products R_{t+1} delta_{t+1}, whose
// partial sums are the next exchange's input. Expanding the update,
//   R_{t+1} delta_{t+1} = R_{t+1} (delta_t - eta mu) - eta (R_{t+1} R_t^T) g_t,
// so the next exchange's partial is P - eta G g_t with P = R_{t+1} (delta_t - eta mu) and the b x b Gram
// block G = R_{t+1} R_t^T of the workgroup's column slice, neither of which needs g_t. They are formed
// while the exchange of step t is in flight, and only the b x b mat-vec G g_t stays between two
// exchanges. The update itself and the averaged snapshot are the same arithmetic as in k_inner.hip.
//
// Workgroup roles (512 threads, one slice of at most 64 columns, b <= 64), one barrier per step:
//  * waves 0-3 hold the slice's delta, running sum and mu (column quad 4 (wave) + lane % 4, rows
//    lane / 4 + 16 q) and the FP32 rows of six steps (gathered four steps ahead); per step they update
//    delta with the previous step's coefficients, form P for the next step and stage the rows of the
//    step after it in LDS as BF16 high and low parts (x = hi + lo + O(2^-16 |x|));
//  * waves 4-7 hold G of the coming step in MFMA accumulators, one 16-row block each (gfx950's 16x16x32
//    BF16 MFMA; hi hi + hi lo + lo hi for FP32 rows, hi hi for BF16 rows, which is exact). After the
//    barrier they form P - eta G g_t for their rows, post it to the other workgroups, then build the
//    next G from LDS;
//  * wave 7 then gathers the W workgroups' words of the step and publishes g_t in LDS.
// The exchange words and their tags are those of k_inner.hip (step t of the epoch is tagged
// step_base + t + 1); step 0 needs no exchange, since delta_0 = 0 makes its dot products zero.
#include "scs_internal.h"

namespace scs {

namespace {

constexpr int kLaThreads = 512;
constexpr uint32_t kLaPollBudget = 1u << 22;
constexpr int kLaSW = 64 + 8;   // BF16 halves per staged row (64 columns and padding)
constexpr int kLaPS = 16 + 4;   // floats per row of the partial-product array

__device__ __forceinline__ void la_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

typedef __attribute__((address_space(1))) const char gchar;
typedef float f32x4_v __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2_v __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) const f32x4_v gf32x4;
typedef __attribute__((address_space(1))) const u32x2_v gu32x2;
typedef __attribute__((address_space(1))) const int32_t gint32;
typedef __attribute__((address_space(1))) const float gfloat;
typedef __attribute__((address_space(1))) uint64_t guint64;
typedef float f4v __attribute__((ext_vector_type(4)));
typedef short s8v __attribute__((ext_vector_type(8)));
typedef float f8v __attribute__((ext_vector_type(8)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

__device__ __forceinline__ float la_get(const float4& v, int i) { return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w; }

// Sum over the 16 lanes of the wave with the same lane % 4 (as in k_inner.hip).
__device__ __forceinline__ float la_rowgroup_sum(float v) {
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x128, 0xf, 0xf, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x124, 0xf, 0xf, false));
  auto p16 = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  v = __uint_as_float(p16[0]) + __uint_as_float(p16[1]);
  auto p32 = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(p32[0]) + __uint_as_float(p32[1]);
}

// Sum over the 16 lanes of each 16-lane row of the wave, left in all of them (DPP row rotations).
__device__ __forceinline__ float la_row16_sum(float v) {
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x128, 0xf, 0xf, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x124, 0xf, 0xf, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x122, 0xf, 0xf, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x121, 0xf, 0xf, false));
  return v;
}

__device__ __forceinline__ f4v la_mfma(const s8v& a, const s8v& b, const f4v& acc) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8v, a), __builtin_bit_cast(bf8v, b), acc, 0, 0,
                                                 0);
}

// Workgroup w of the inner loop. RPT: row groups per thread (b <= 16 RPT).
template <int RPT, bool BF16>
__device__ __forceinline__ void inner_la_body(const InnerArgs& a, const int w) {
  constexpr int ES = BF16 ? 2 : 4;
  constexpr int RB = 16 * RPT;      // rows of a step (b <= RB)
  constexpr int NPL = BF16 ? 1 : 2; // BF16 planes staged per row: high, and low for FP32 rows
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const bool dwave = wave < 4;
  const bool xwave = wave == 7;
  const int gb = wave - 4;          // Gram row block of waves 4-7
  const bool hasblk = wave >= 4 && gb < RPT;
  const int rg = lane >> 2;
  const int cgt = 4 * (wave & 3) + (lane & 3);   // column quad of a data thread
  const int b = a.b, W = a.W;
  const uint32_t NR = (uint32_t)(a.n + a.d), n32 = (uint32_t)a.n;
  const int64_t c_begin = (int64_t)w * a.slice;
  const int64_t c_end = c_begin + a.slice < a.d ? c_begin + a.slice : a.d;
  const int64_t m = a.m, mlast = a.m - 1;
  guint64* xb = (guint64*)a.xbuf;
  const gint32* gidx = (const gint32*)a.idx;
  const gfloat* gscale = (const gfloat*)a.scale;
  const char* xt_base = reinterpret_cast<const char*>(a.Xt);
  const char* reg_base =
      reinterpret_cast<const char*>((uintptr_t)a.reg - (uintptr_t)a.n * (uintptr_t)a.ldx * (uintptr_t)ES);
  const uint64_t ldb = (uint64_t)a.ldx * ES;

  __shared__ __align__(16) uint16_t s_bf[3][NPL][RB * kLaSW];   // BF16 parts of the rows of three steps
  __shared__ __align__(16) float s_p[2][RB * kLaPS];            // P of a step per row and column quad
  __shared__ __align__(16) float s_gam[2][RB];                  // coefficients g_t (by step parity)
  __shared__ int s_abort;
  __shared__ int s_posted;   // Gram waves that have posted, summed over the steps

  // data threads: the column quad and its state
  const int64_t col = c_begin + 4 * cgt;
  const bool cin = dwave && col < c_end;
  const uint64_t colb = (uint64_t)(cin ? col : 0) * ES;
  bool cok[4];
  float dl[4], sm[4], smc[4], muv[4], w0[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    cok[v] = dwave && col + v < c_end;
    muv[v] = cok[v] ? a.mu[col + v] : 0.f;
    w0[v] = cok[v] ? a.wt[col + v] : 0.f;
    dl[v] = 0.f;
    sm[v] = 0.f;
    smc[v] = 0.f;
  }
  const float eta = a.eta_from_state
                        ? (float)ldexp(a.step_scale * (double)a.n / a.state->beta_sum, -a.state->backoffs)
                        : (float)a.eta;
  if (tid == 0) {
    s_abort = 0;
    s_posted = 0;
  }
  const int nposting = RPT;   // Gram waves with rows to post

  // index of row q of step s for this data thread (rows past b repeat row b - 1; their coefficient is 0)
  auto load_index = [&](int64_t s, int32_t (&ix)[RPT]) {
    const int64_t ss = s < mlast ? s : mlast;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int j = rg + 16 * q;
      ix[q] = gidx[ss * b + (j < b ? j : b - 1)];
    }
  };
  // loads of a step's rows (every data thread issues the same loads; out-of-slice columns read a fixed
  // in-bounds address), zeroed outside the slice when used
  auto load_rows = [&](const int32_t (&ix)[RPT], float4 (&buf)[RPT]) {
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const uint32_t i = (uint32_t)ix[q] < NR ? (uint32_t)ix[q] : 0u;
      const gchar* rowp = (const gchar*)((i < n32 ? xt_base : reg_base) + (uint64_t)i * ldb);
      const gchar* p = cin ? rowp + colb : (const gchar*)xt_base;
      if constexpr (BF16) {
        const u32x2_v u = *reinterpret_cast<const gu32x2*>(p);
        buf[q] = make_float4(__uint_as_float(u[0] << 16), __uint_as_float(u[0] & 0xffff0000u),
                             __uint_as_float(u[1] << 16), __uint_as_float(u[1] & 0xffff0000u));
      } else {
        const f32x4_v x = *reinterpret_cast<const gf32x4*>(p);
        buf[q] = make_float4(x[0], x[1], x[2], x[3]);
      }
    }
  };
  auto masked = [&](const float4& x) {
    return make_float4(cok[0] ? x.x : 0.f, cok[1] ? x.y : 0.f, cok[2] ? x.z : 0.f, cok[3] ? x.w : 0.f);
  };
  // a step's rows into its LDS slot as BF16 high (and low) parts; the registers keep the rows with the
  // columns outside the slice zeroed, as the update and P use them
  auto stage_rows = [&](int64_t step, float4 (&buf)[RPT]) {
    const int sl = (int)(step % 3);
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const float4 x = masked(buf[q]);
      buf[q] = x;
      const int off = (rg + 16 * q) * kLaSW + 4 * cgt;
      const uint32_t h0 = pack_bf16x2(x.x, x.y), h1 = pack_bf16x2(x.z, x.w);
      *reinterpret_cast<uint2*>(&s_bf[sl][0][off]) = make_uint2(h0, h1);
      if constexpr (!BF16) {
        const uint32_t l0 = pack_bf16x2(x.x - __uint_as_float(h0 << 16), x.y - __uint_as_float(h0 & 0xffff0000u));
        const uint32_t l1 = pack_bf16x2(x.z - __uint_as_float(h1 << 16), x.w - __uint_as_float(h1 & 0xffff0000u));
        *reinterpret_cast<uint2*>(&s_bf[sl][NPL - 1][off]) = make_uint2(l0, l1);
      }
    }
  };
  // delta <- delta - eta (R^T g + mu) with rows R of one step and its coefficients g (in s_gam[par]),
  // then the compensated running sum
  auto update = [&](const float4 (&Rr)[RPT], int par) {
    float u[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const float g8 = s_gam[par][rg + 16 * q];
      const float4 x = Rr[q];
#pragma unroll
      for (int v = 0; v < 4; ++v) u[v] = fmaf(g8, la_get(x, v), u[v]);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float g = cok[v] ? la_rowgroup_sum(u[v]) : 0.f;
      dl[v] -= eta * (g + muv[v]);
      const float y = dl[v] - smc[v];
      const float s2 = sm[v] + y;
      smc[v] = (s2 - sm[v]) - y;
      sm[v] = s2;
    }
  };

  bool go = true;
  if (dwave) {
    // ---- data waves. Set k of the six-set ring holds step s with s = k - 1 (mod 6); window t uses the
    // sets of steps t - 1 (update), t + 1 (P), t + 2 (staged) and loads step t + 4; indices rotate by 3.
    float4 R[6][RPT];
    int32_t I[3][RPT];
    load_index(0, I[0]);
    load_index(1, I[1]);
    load_rows(I[0], R[1]);
    load_rows(I[1], R[2]);
    load_index(2, I[0]);
    load_index(3, I[1]);
    stage_rows(0, R[1]);
    stage_rows(1, R[2]);
    load_rows(I[0], R[3]);   // step 2
    load_rows(I[1], R[4]);   // step 3
    load_index(4, I[2]);
    la_barrier();   // staged rows of steps 0 and 1 are visible
    auto dwindow = [&](int64_t t, float4 (&Rm1)[RPT], float4 (&Rp1)[RPT], float4 (&Rp2)[RPT], float4 (&Rp4)[RPT],
                       int32_t (&Iu)[RPT], int32_t (&In)[RPT]) -> bool {
      // step t + 5's indices, then step t + 4's rows: both consumed a window later or more
      load_index(t + 5, In);
      load_rows(Iu, Rp4);
      if (t >= 1) update(Rm1, (int)((t - 1) & 1));
      if (t + 1 < m) {
        // P_{t+1} = R_{t+1} (delta_t - eta mu) over this thread's four columns
        float dm[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) dm[v] = dl[v] - eta * muv[v];
        float* dst = s_p[(t + 1) & 1];
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          const float4 x = Rp1[q];
          float p = 0.f;
#pragma unroll
          for (int v = 0; v < 4; ++v) p = fmaf(la_get(x, v), dm[v], p);
          dst[(rg + 16 * q) * kLaPS + cgt] = p;
        }
      }
      if (t + 2 < m) stage_rows(t + 2, Rp2);
      la_barrier();
      return !s_abort;
    };
    int64_t t = 0;
    for (; go && t + 5 < m; t += 6) {
      go = dwindow(t, R[0], R[2], R[3], R[5], I[2], I[0]) && dwindow(t + 1, R[1], R[3], R[4], R[0], I[0], I[1]) &&
           dwindow(t + 2, R[2], R[4], R[5], R[1], I[1], I[2]) && dwindow(t + 3, R[3], R[5], R[0], R[2], I[2], I[0]) &&
           dwindow(t + 4, R[4], R[0], R[1], R[3], I[0], I[1]) && dwindow(t + 5, R[5], R[1], R[2], R[4], I[1], I[2]);
    }
    if (go && t < m) go = dwindow(t, R[0], R[2], R[3], R[5], I[2], I[0]);
    if (go && t + 1 < m) go = dwindow(t + 1, R[1], R[3], R[4], R[0], I[0], I[1]);
    if (go && t + 2 < m) go = dwindow(t + 2, R[2], R[4], R[5], R[1], I[1], I[2]);
    if (go && t + 3 < m) go = dwindow(t + 3, R[3], R[5], R[0], R[2], I[2], I[0]);
    if (go && t + 4 < m) go = dwindow(t + 4, R[4], R[0], R[1], R[3], I[0], I[1]);
    if (go) {
      // the last update, with step m - 1 (set m % 6) and its coefficients
      const int sl = (int)(m % 6);
      float4 Rl[RPT];
#pragma unroll
      for (int q = 0; q < RPT; ++q) Rl[q] = R[0][q];
#pragma unroll
      for (int k6 = 1; k6 < 6; ++k6)
        if (k6 == sl)
#pragma unroll
          for (int q = 0; q < RPT; ++q) Rl[q] = R[k6][q];
      update(Rl, (int)((m - 1) & 1));
      if (rg == 0) {   // lanes 0..3: one writer per column quad
        const float inv_m = 1.0f / (float)m;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t c = col + v;
          if (cok[v]) {
            if (a.wt_prev) a.wt_prev[c] = w0[v];
            const float upd = a.average ? (sm[v] - smc[v]) * inv_m : dl[v];
            a.wt[c] = w0[v] + upd;
          }
        }
      }
    }
  } else {
    // ---- waves 4-7: acc holds G_{t,t-1} for the rows of block gb against all rows; wave 7 also gathers
    // the exchange (lane j < b: row j's W words) and publishes g_t
    const int r = lane & 15, g = lane >> 4;
    f4v acc[RPT];
    auto gram = [&](int64_t t1) {   // G_{t1, t1 - 1}
      const uint16_t* sa[NPL];
      const uint16_t* sb[NPL];
#pragma unroll
      for (int pl = 0; pl < NPL; ++pl) {
        sa[pl] = s_bf[t1 % 3][pl];
        sb[pl] = s_bf[(t1 - 1) % 3][pl];
      }
#pragma unroll
      for (int jb = 0; jb < RPT; ++jb) acc[jb] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < 2; ++kb) {
        const int ao = (16 * gb + r) * kLaSW + 32 * kb + 8 * g;
        const s8v ah = *reinterpret_cast<const s8v*>(&sa[0][ao]);
        s8v al;
        if constexpr (!BF16) al = *reinterpret_cast<const s8v*>(&sa[NPL - 1][ao]);
#pragma unroll
        for (int jb = 0; jb < RPT; ++jb) {
          const int bo = (16 * jb + r) * kLaSW + 32 * kb + 8 * g;
          const s8v bh = *reinterpret_cast<const s8v*>(&sb[0][bo]);
          acc[jb] = la_mfma(ah, bh, acc[jb]);
          if constexpr (!BF16) {
            const s8v bl = *reinterpret_cast<const s8v*>(&sb[NPL - 1][bo]);
            acc[jb] = la_mfma(ah, bl, acc[jb]);
            acc[jb] = la_mfma(al, bh, acc[jb]);
          }
        }
      }
    };
    const bool xrow = xwave && lane < b;
    float sc_next = 0.f;
    if (xwave) {
      if (lane < RB) s_gam[0][lane] = 0.f;   // g_0 = 0: delta_0 = 0
      sc_next = gscale[(1 < mlast ? 1 : mlast) * b + (lane < b ? lane : b - 1)];   // step 1's weights
    }
    la_barrier();   // rows of steps 0 and 1 are staged
    if (hasblk && 1 < m) gram(1);
    la_barrier();   // end of window 0 (P_1 is in LDS)
    if (s_abort) go = false;
    for (int64_t t = 1; go && t < m; ++t) {
      const int par = (int)(t & 1);
      const uint32_t target = a.step_base + (uint32_t)t + 1u;
      if (hasblk) {
        // Q_j = P_t[j] - eta (G_{t,t-1} g_{t-1})_j for the rows of block gb, posted as step t's word.
        // acc[jb][k] = G[16 gb + 4 g + k][16 jb + r]: sum over jb with g_{t-1}[16 jb + r], then over r
        const float* gp = s_gam[(t - 1) & 1];
        const float* pp = s_p[t & 1];
        float y[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int jb = 0; jb < RPT; ++jb) {
          const float gv = gp[16 * jb + r];
#pragma unroll
          for (int k = 0; k < 4; ++k) y[k] = fmaf(acc[jb][k], gv, y[k]);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) y[k] = la_row16_sum(y[k]);
        // lane (r < 4, g) posts row 16 gb + 4 g + r
        const int row = 16 * gb + 4 * g + (r & 3);
        const float yv = (r & 3) == 0 ? y[0] : (r & 3) == 1 ? y[1] : (r & 3) == 2 ? y[2] : y[3];
        if (r < 4 && row < b) {
          float q = 0.f;
#pragma unroll
          for (int c = 0; c < 16; c += 4) {
            const float4 v4 = *reinterpret_cast<const float4*>(&pp[row * kLaPS + c]);
            q += (v4.x + v4.y) + (v4.z + v4.w);
          }
          q = fmaf(-eta, yv, q);
          guint64* slot = xb + ((int64_t)par * W) * 64;
          __hip_atomic_store(&slot[(int64_t)w * 64 + row], ((uint64_t)target << 32) | __float_as_uint(q),
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (lane == 0) atomicAdd(&s_posted, 1);
        // the next step's G, while the exchange is in flight
        if (t + 1 < m) gram(t + 1);
      }
      if (xwave) {
        const float scl = sc_next;
        sc_next = gscale[(t + 1 < mlast ? t + 1 : mlast) * b + (lane < b ? lane : b - 1)];
        // the posts of this step come after the Gram waves' mat-vecs: wait for this workgroup's, then
        // about 0.1 us (the other workgroups post at about the same time; earlier polls only return stale
        // words and slow the posts down)
        for (uint32_t spin = 0; spin < (1u << 20); ++spin)
          if (__hip_atomic_load(&s_posted, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >= nposting * (int)t) break;
        __builtin_amdgcn_s_sleep(4);
        guint64* slot = xb + ((int64_t)par * W) * 64 + lane;
        uint64_t xv[16];
#pragma unroll
        for (int v = 0; v < 16; ++v)
          xv[v] = (v < W && xrow) ? __hip_atomic_load(&slot[v * 64], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                  : ((uint64_t)target << 32);
        uint32_t polls = 0;
        bool bad = false;
        for (;;) {
          bool pending = false;
#pragma unroll
          for (int v = 0; v < 16; ++v) pending |= (uint32_t)(xv[v] >> 32) != target;
          if (!pending) break;
          if ((++polls & 1023u) == 0 &&
              (polls > kLaPollBudget ||
               __hip_atomic_load(&a.state->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == SCS_EDEVICE)) {
            bad = true;
            break;
          }
#pragma unroll
          for (int v = 0; v < 16; ++v)
            if ((uint32_t)(xv[v] >> 32) != target)
              xv[v] = __hip_atomic_load(&slot[v * 64], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (__any(bad) && lane == 0) {
          s_abort = 1;
          __hip_atomic_store(&a.state->status, SCS_EDEVICE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(&a.state->done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        float cl = 0.f;
#pragma unroll
        for (int v = 0; v < 16; ++v)
          if (v < W) cl += __uint_as_float((uint32_t)xv[v]);  // same order in every workgroup
        if (lane < RB) s_gam[par][lane] = xrow ? scl * cl / (float)b : 0.f;
      }
      la_barrier();
      if (s_abort) go = false;
    }
  }
  if (go && w == 0 && tid == 0) {
    a.state->epochs += 1;
    a.state->eta = (double)eta;
  }
}

template <int RPT, bool BF16>
__global__ __launch_bounds__(kLaThreads) void inner_la_kernel(InnerArgs a) {
  const int bid = blockIdx.x;
  if (bid % a.xcd_stride != 0) return;
  const int w = bid / a.xcd_stride;
  if (w >= a.W) return;
  if (a.state->done) return;
  inner_la_body<RPT, BF16>(a, w);
}

template <int RPT, bool BF16>
int launch_la(hipStream_t st, InnerArgs& a) {
  dim3 grid((unsigned)(a.W * a.xcd_stride)), block(kLaThreads);
  inner_la_kernel<RPT, BF16><<<grid, block, 0, st>>>(a);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

}  // namespace

bool inner_lookahead_fits(int b, int64_t d, int W) {
  const int64_t slice = cdiv(cdiv(d, W), 4) * 4;
  return b >= 1 && b <= 64 && slice <= 64 && W >= 1 && W <= 16;
}

int launch_inner_epoch_lookahead(hipStream_t st, InnerArgs& a, int bf16) {
  if (a.m < 1 || !inner_lookahead_fits(a.b, a.d, a.W)) {
    set_error("look-ahead inner loop: needs 1 <= b <= 64, at most 64 columns per workgroup, 1 <= workgroups <= 16");
    return SCS_EINVAL;
  }
  if (a.ldx % 4 != 0 || a.ldr != a.ldx) {
    set_error("inner loop: data and regularizer rows need one leading dimension, a multiple of 4");
    return SCS_EINVAL;
  }
  a.slice = cdiv(cdiv(a.d, a.W), 4) * 4;
  const int rpt = a.b <= 16 ? 1 : a.b <= 32 ? 2 : 4;
  if (bf16) {
    if (rpt == 1) return launch_la<1, true>(st, a);
    if (rpt == 2) return launch_la<2, true>(st, a);
    return launch_la<4, true>(st, a);
  }
  if (rpt == 1) return launch_la<1, false>(st, a);
  if (rpt == 2) return launch_la<2, false>(st, a);
  return launch_la<4, false>(st, a);
}

}  // namespace scs
