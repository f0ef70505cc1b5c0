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
// slice of delta, mu and sum in registers (replicated over its row groups) and gathers only
// its slice of the b rows. The b partial dot products of a step are exchanged through global
// memory: every workgroup posts its partials and a step counter, then sums all W partials in
// the same fixed order, so all workgroups compute bit-identical c_j. Waits are bounded: a wait
// that exceeds its poll budget raises an abort flag that ends every workgroup's loop.
// Rows of the next step are loaded while the current step's reductions run (the index stream
// does not depend on the iterate).
#include <type_traits>

#include "scs_internal.h"

namespace scs {



namespace {

constexpr int kInnerThreads = 512;  // 8 waves
constexpr uint32_t kPollBudget = 1u << 22;

// Barrier for LDS traffic only: waits for this wave's LDS operations but not for its
// outstanding global loads (the prefetched rows of the next step stay in flight).
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }


typedef __attribute__((address_space(1))) const char gchar;
typedef float f32x4_v __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2_v __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) const f32x4_v gf32x4;
typedef __attribute__((address_space(1))) const u32x2_v gu32x2;
typedef __attribute__((address_space(1))) const int32_t gint32;
typedef __attribute__((address_space(1))) const float gfloat;
typedef __attribute__((address_space(1))) uint64_t guint64;

__device__ __forceinline__ float f4get(const float4& v, int i) { return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w; }

// Sum of v over the 16 lanes of the wave with the same lane % 4 (the 16 row groups sharing a
// column), left in every one of them: DPP rotations by 8 and 4 inside each 16-lane row, then the
// gfx950 row swaps, which exchange 16-lane rows 0<->1, 2<->3 and 32-lane halves respectively.
__device__ __forceinline__ float rowgroup_sum(float v) {
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x128, 0xf, 0xf, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x124, 0xf, 0xf, false));
  auto p16 = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  v = __uint_as_float(p16[0]) + __uint_as_float(p16[1]);
  auto p32 = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(p32[0]) + __uint_as_float(p32[1]);
}

// Layout: the workgroup's 8 waves form WR wave-rows of WC = 8 / WR waves. A wave-row owns 16 RPT
// of the step's b rows (rows j = r0 + rg + 16 q, r0 = 16 RPT * wave-row) over all of the
// workgroup's columns, so larger minibatches spread over more waves instead of more registers.
// Inside a wave, lane = 4 * rg + cl: the 16 row groups that share a column are in one wave and a
// sum over them is a lane butterfly; column thread cgt = 4 * (wave % WC) + cl owns columns
// c_begin + 4 (cgt + 4 WC q) .. + 3 for q < CPT.
// The first wave of each wave-row owns that wave-row's per-step communication: it sums the partial
// dot products of its rows, exchanges them with the other workgroups, publishes the step
// coefficients and stages its rows' indices into LDS two steps ahead, so the exchanges of the
// wave-rows run side by side. With WR > 1 the update's sum over rows ends with one LDS round trip
// that adds the wave-rows' sums in a fixed order (every wave-row then holds the same delta).
// Every global load a wave issues is consumed at least one step later, except the exchange polls,
// so no wait for one load also waits for a load issued after it (loads complete in order per
// wave). Rows live in a two-slot ring whose roles alternate at compile time. Data rows and
// regularizer rows share one leading dimension, so a row address is one multiply-add from a base
// selected by the index range.
// Workgroup w (0 <= w < a.W) of one problem's inner loop.
template <int RPT, int CPT, int WR, bool BF16>
__device__ __forceinline__ void inner_epoch_body(const InnerArgs& a, const int w) {
  constexpr int ES = BF16 ? 2 : 4;          // bytes per element
  constexpr int WC = 8 / WR;                // waves per wave-row
  constexpr int CT = 4 * WC;                // column threads per wave-row
  constexpr int RW = 16 * RPT;              // rows per wave-row
  constexpr int PDS = CT + 4;               // row stride of the partial-dot array (floats)
  constexpr int CS = 4 * CT * CPT;          // columns a wave-row covers
  const int tid = threadIdx.x, lane = tid & 63;
  // wave index made provably uniform so that wave-row and exchange-wave tests are scalar branches
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave / WC;
  const bool ldwave = wave % WC == 0;       // this wave stages its wave-row's indices and weights
  const int r0 = wr * RW;
  const int rg = lane >> 2;                 // row group
  const int cgt = (wave % WC) * 4 + (lane & 3);
  const int b = a.b, W = a.W;
  const uint32_t NR = (uint32_t)(a.n + a.d), n32 = (uint32_t)a.n;
  const int64_t c_begin = (int64_t)w * a.slice;
  const int64_t c_end = c_begin + a.slice < a.d ? c_begin + a.slice : a.d;
  const int64_t mlast = a.m - 1;
  // the pointers used every step are in the global address space, so their loads are not flat loads
  // (which an LDS barrier's wait would also wait for)
  guint64* xb = (guint64*)a.xbuf;
  const gint32* gidx = (const gint32*)a.idx;
  const gfloat* gscale = (const gfloat*)a.scale;
  const char* xt_base = reinterpret_cast<const char*>(a.Xt);
  // base for regularizer rows, offset so that row i >= n is at reg_base + i * ld (pointer arithmetic
  // done on integers; only ever dereferenced for i >= n)
  const char* reg_base =
      reinterpret_cast<const char*>((uintptr_t)a.reg - (uintptr_t)a.n * (uintptr_t)a.ldx * (uintptr_t)ES);
  const uint64_t ldb = (uint64_t)a.ldx * ES;

  __shared__ __align__(16) float pd[WR * RW * PDS];
  __shared__ float gam[WR * RW];
  __shared__ __align__(16) int32_t s_idx[4][WR][16][4];  // [step slot][wave-row][row group][q]
  __shared__ float s_sc[2][WR * RW];                       // weights 1/(n q_i) of the rows of two steps
  __shared__ __align__(16) float red[WR > 1 ? WR : 1][WR > 1 ? CS : 4];
  __shared__ int s_abort;

  float dl[CPT][4], sm[CPT][4], smc[CPT][4], muv[CPT][4], w0[CPT][4];
  int64_t col[CPT];
  uint64_t colb[CPT];   // byte offset of the 4 columns loaded (inside the slice, a multiple of 4)
  bool cin[CPT];        // the column group starts inside the slice
  bool cok[CPT][4];
#pragma unroll
  for (int q = 0; q < CPT; ++q) {
    col[q] = c_begin + 4 * (cgt + CT * q);
    // column groups past the slice (or past d, for a workgroup whose slice starts beyond the last
    // column) all load the first 16 bytes of the first data row, which stay in the CU's cache; their
    // values are masked out by cok
    cin[q] = col[q] < c_end;
    colb[q] = (uint64_t)(cin[q] ? col[q] : 0) * ES;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      int64_t c = col[q] + v;
      cok[q][v] = c < c_end;
      muv[q][v] = cok[q][v] ? a.mu[c] : 0.f;
      w0[q][v] = cok[q][v] ? a.wt[c] : 0.f;
      dl[q][v] = 0.f;
      sm[q][v] = 0.f;
      smc[q][v] = 0.f;
    }
  }
  const float eta = a.eta_from_state
                        ? (float)ldexp(a.step_scale * (double)a.n / a.state->beta_sum, -a.state->backoffs)
                        : (float)a.eta;
  if (tid == 0) s_abort = 0;

  // Row loads are unconditional from in-bounds addresses: rows j >= b get coefficient 0 and
  // columns outside the slice are zeroed before use.
  // Row loads go through global-address-space pointers: a generic (flat) load would also count as an
  // LDS operation, and every LDS barrier's wait would then wait for the rows prefetched for the next step.
  auto load_rows = [&](int slot, float4 (&buf)[RPT][CPT]) {
    const int4 i0 = *reinterpret_cast<const int4*>(&s_idx[slot][wr][rg][0]);
    const int32_t ix[4] = {i0.x, i0.y, i0.z, i0.w};
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const uint32_t i = (uint32_t)ix[q] < NR ? (uint32_t)ix[q] : 0u;
      const gchar* rowp = (const gchar*)((i < n32 ? xt_base : reg_base) + (uint64_t)i * ldb);
#pragma unroll
      for (int c = 0; c < CPT; ++c) {
        const gchar* p = cin[c] ? rowp + colb[c] : (const gchar*)xt_base;
        if constexpr (BF16) {
          const u32x2_v u = *reinterpret_cast<const gu32x2*>(p);
          buf[q][c] = make_float4(__uint_as_float(u[0] << 16), __uint_as_float(u[0] & 0xffff0000u),
                                  __uint_as_float(u[1] << 16), __uint_as_float(u[1] & 0xffff0000u));
        } else {
          const f32x4_v x = *reinterpret_cast<const gf32x4*>(p);
          buf[q][c] = make_float4(x[0], x[1], x[2], x[3]);
        }
      }
    }
  };

  // The exchange of a wave-row's partial sums runs in a wave with no column of the slice when the
  // wave-row has one (its row loads all hit the cache, so its polls, which complete in order after
  // them, do not wait for rows gathered from memory), else in the wave-row's first wave.
  const bool xwave = (wave % WC) == ((int64_t)16 * (WC - 1) >= c_end - c_begin ? WC - 1 : 0);
  // Lane j of the exchange and staging waves serves row r0 + j of the step (j < RW); jj clamps it to a
  // drawn row
  const int myrow = r0 + lane;
  const bool rowok = lane < RW && myrow < b;
  const int jj = rowok ? myrow : b - 1;
  const int srg = lane & 15, sq = lane >> 4;  // where lane j stages its row's index (j = srg + 16 sq)
  // Staging waves, two-slot rings alternating like the row buffers: step t stages idxX (index of step
  // t+2) and scX (weight of step t+1), both loaded one step earlier together with the rows, and loads
  // the other slot
  int32_t idxA = 0, idxB = 0;
  float scA = 0.f, scB = 0.f;
  if (ldwave) {
    s_idx[0][wr][srg][sq] = rowok ? gidx[jj] : 0;
    s_idx[1][wr][srg][sq] = rowok ? gidx[(1 < mlast ? 1 : mlast) * b + jj] : 0;
    if (lane < RW) s_sc[0][myrow] = gscale[jj];
  }
  idxA = gidx[(2 < mlast ? 2 : mlast) * b + jj];
  scA = gscale[(1 < mlast ? 1 : mlast) * b + jj];
  float4 bufA[RPT][CPT], bufB[RPT][CPT];
  lds_barrier();
  load_rows(0, bufA);

  // One inner step t on rows `cur`, prefetching the rows of step t+1 into `nxt`.
  // Returns false when the epoch must stop (abort).
  auto step = [&](int64_t t, float4 (&cur)[RPT][CPT], float4 (&nxt)[RPT][CPT], int32_t& idx_use, int32_t& idx_next,
                  float& sc_use, float& sc_next) -> bool {
    load_rows((int)((t + 1) & 3), nxt);
    // consumed at the next step, queued behind this step's row loads. Every wave issues them (only the
    // staging wave uses them; the others hit the cache): with the same loads in flight in every wave,
    // the compiler's count of outstanding loads is exact, and the wait for this step's rows does not
    // also wait for the rows just prefetched.
    idx_next = gidx[(t + 3 < mlast ? t + 3 : mlast) * b + jj];
    sc_next = gscale[(t + 2 < mlast ? t + 2 : mlast) * b + jj];
    // columns outside the slice (and padding past d) may hold anything: zero them, then partial
    // dot products over this workgroup's columns
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
#pragma unroll
      for (int c = 0; c < CPT; ++c) {
        cur[q][c].x = cok[c][0] ? cur[q][c].x : 0.f;
        cur[q][c].y = cok[c][1] ? cur[q][c].y : 0.f;
        cur[q][c].z = cok[c][2] ? cur[q][c].z : 0.f;
        cur[q][c].w = cok[c][3] ? cur[q][c].w : 0.f;
      }
      float p = 0.f;
#pragma unroll
      for (int c = 0; c < CPT; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) p = fmaf(f4get(cur[q][c], v), dl[c][v], p);
      pd[(r0 + rg + 16 * q) * PDS + cgt] = p;
    }
    if (ldwave) {
      s_idx[(t + 2) & 3][wr][srg][sq] = rowok ? idx_use : 0;
      if (lane < RW) s_sc[(t + 1) & 1][myrow] = sc_use;
    }
    lds_barrier();
    if (xwave) {
      float cl = 0.f;
      const float scl = lane < RW ? s_sc[t & 1][myrow] : 0.f;  // read before the exchange, used after it
      if (lane < RW) {
#pragma unroll
        for (int g = 0; g < CT; g += 4) {
          const float4 v4 = *reinterpret_cast<const float4*>(&pd[myrow * PDS + g]);
          cl += (v4.x + v4.y) + (v4.z + v4.w);
        }
      }
      if (W > 1) {
        // post (step tag, value) as one 64-bit word; gather the W words of this row; a word is
        // valid once its tag is this step's, so no fence is needed
        const int par = (int)(t & 1);
        const uint32_t target = a.step_base + (uint32_t)t + 1u;
        // words of (parity, wave-row, workgroup v) in blocks of 64 rows: a lane's W words are 512 bytes
        // apart, which spreads them over the cache channels
        guint64* slot = xb + ((int64_t)(par * WR + wr) * W) * 64 + lane;
        const bool xrow = lane < RW;
        if (xrow)
          __hip_atomic_store(&slot[(int64_t)w * 64], ((uint64_t)target << 32) | __float_as_uint(cl),
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // first poll about 0.2 us (512 cycles) after the post: polls issued at once mostly return
        // stale words and slow the posts of the other workgroups down (measured: 2.33 -> 1.94 us per
        // step at 16 workgroups, b = 64; 2.42 -> 2.05 at 8)
        __builtin_amdgcn_s_sleep(8);
        uint64_t xv[16];
#pragma unroll
        for (int v = 0; v < 16; ++v)
          xv[v] = (v < W && xrow)
                      ? __hip_atomic_load(&slot[v * 64], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                      : ((uint64_t)target << 32);
        uint32_t polls = 0;
        bool bad = false;
        for (;;) {
          bool pending = false;
#pragma unroll
          for (int v = 0; v < 16; ++v) pending |= (uint32_t)(xv[v] >> 32) != target;
          if (!pending) break;
          if ((++polls & 1023u) == 0 &&
              (polls > kPollBudget ||
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
        float sum = 0.f;
#pragma unroll
        for (int v = 0; v < 16; ++v)
          if (v < W) sum += __uint_as_float((uint32_t)xv[v]);  // same order in every workgroup
        cl = sum;
      }
      if (lane < RW) gam[myrow] = rowok ? scl * cl / (float)b : 0.f;
    }
    lds_barrier();
    if (s_abort) return false;
    // (1/b) sum_j c_j a_j / (n q_j): this thread's rows, then the 16 row groups of the wave, then
    // (WR > 1) the wave-rows in order
    float g8[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) g8[q] = gam[r0 + rg + 16 * q];
    float uu[CPT][4];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      float u[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int q = 0; q < RPT; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) u[v] = fmaf(g8[q], f4get(cur[q][c], v), u[v]);
#pragma unroll
      for (int v = 0; v < 4; ++v) uu[c][v] = rowgroup_sum(u[v]);
    }
    if constexpr (WR > 1) {
      if (rg == 0) {
#pragma unroll
        for (int c = 0; c < CPT; ++c)
          *reinterpret_cast<float4*>(&red[wr][4 * (cgt + CT * c)]) =
              make_float4(uu[c][0], uu[c][1], uu[c][2], uu[c][3]);
      }
      lds_barrier();
#pragma unroll
      for (int c = 0; c < CPT; ++c) {
        float4 s4 = *reinterpret_cast<const float4*>(&red[0][4 * (cgt + CT * c)]);
#pragma unroll
        for (int r = 1; r < WR; ++r) {
          const float4 o4 = *reinterpret_cast<const float4*>(&red[r][4 * (cgt + CT * c)]);
          s4.x += o4.x;
          s4.y += o4.y;
          s4.z += o4.z;
          s4.w += o4.w;
        }
        uu[c][0] = s4.x;
        uu[c][1] = s4.y;
        uu[c][2] = s4.z;
        uu[c][3] = s4.w;
      }
    }
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float g = cok[c][v] ? uu[c][v] : 0.f;
        dl[c][v] -= eta * (g + muv[c][v]);
        float y = dl[c][v] - smc[c][v];
        float s2 = sm[c][v] + y;
        smc[c][v] = (s2 - sm[c][v]) - y;
        sm[c][v] = s2;
      }
    }
    return true;
  };

  int64_t t = 0;
  bool go = true;
  for (; go && t + 1 < a.m; t += 2)
    go = step(t, bufA, bufB, idxA, idxB, scA, scB) && step(t + 1, bufB, bufA, idxB, idxA, scB, scA);
  if (go && t < a.m) go = step(t, bufA, bufB, idxA, idxB, scA, scB);

  if (!s_abort && wr == 0 && rg == 0) {  // lanes 0..3 of the first wave-row: one writer per column thread
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

template <int RPT, int CPT, int WR, bool BF16>
__global__ __launch_bounds__(kInnerThreads) void inner_epoch_kernel(InnerArgs a) {
  const int bid = blockIdx.x;
  if (bid % a.xcd_stride != 0) return;
  const int w = bid / a.xcd_stride;
  if (w >= a.W) return;
  if (a.state->done) return;
  inner_epoch_body<RPT, CPT, WR, BF16>(a, w);
}

// All problems of a batch: block w * nprob + p is workgroup w of problem p (with nprob a multiple
// of 8 the W workgroups of a problem share an XCD). The epoch's index stream is slot `slot` of the
// problem's sampled group.
template <int RPT, int CPT, int WR, bool BF16>
__global__ __launch_bounds__(kInnerThreads) void inner_epoch_batched_kernel(const BatchProb* P, int nprob, int slot,
                                                                            int64_t epoch, const int* clk) {
  if (clk) {  // epochs replayed from a graph: the epoch number is on the device
    if (clk[0] >= clk[1]) return;
    epoch = clk[0];
    slot = clk[0] % kEpochGroup;
  }
  const int p = blockIdx.x % nprob, w = blockIdx.x / nprob;
  InnerArgs a = P[p].inner;
  if (w >= a.W || a.state->done) return;
  a.idx = P[p].idx + slot * P[p].draws;
  a.scale = P[p].scale + slot * P[p].draws;
  a.step_base = (uint32_t)((uint64_t)epoch * (uint64_t)a.m);
  inner_epoch_body<RPT, CPT, WR, BF16>(a, w);
}

template <int RPT, int CPT, int WR, bool BF16>
int launch_bt(hipStream_t st, const BatchProb* P, int nprob, int W, int slot, int64_t epoch, const int* clk) {
  dim3 block(kInnerThreads);
  if (W > 1) {
    // The workgroups of a problem wait on each other, so they must all be resident: problems go in
    // groups that fit the device at once, one launch per group (ordinary launches: the stream runs
    // nothing else meanwhile, every group fits the idle device, and every wait is bounded).
    // co-resident workgroups of this instantiation, per device (computed on first use on each)
    constexpr int kMaxDevices = 64;
    static int resident_per_dev[kMaxDevices] = {};
    int dev = 0;
    SCS_HIP(hipGetDevice(&dev));
    int resident = dev < kMaxDevices ? resident_per_dev[dev] : 0;
    if (resident == 0) {
      int per_cu = 0, cus = 0;
      SCS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, (const void*)inner_epoch_batched_kernel<RPT, CPT, WR, BF16>, kInnerThreads, 0));
      SCS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
      resident = per_cu * cus;
      if (dev < kMaxDevices) resident_per_dev[dev] = resident;
    }
    int group = resident / W;
    if (group >= 8) group -= group % 8;  // keeps the W workgroups of a problem on one XCD
    if (group < 1) {
      set_error("batched inner loop: not enough resident workgroups for one problem");
      return SCS_EINVAL;
    }
    for (int p0 = 0; p0 < nprob; p0 += group) {
      const BatchProb* Pg = P + p0;
      int cnt = nprob - p0 < group ? nprob - p0 : group;
      inner_epoch_batched_kernel<RPT, CPT, WR, BF16><<<dim3((unsigned)(cnt * W)), block, 0, st>>>(Pg, cnt, slot, epoch,
                                                                                                   clk);
      SCS_HIP(hipGetLastError());
    }
  } else {
    dim3 grid((unsigned)nprob);
    inner_epoch_batched_kernel<RPT, CPT, WR, BF16><<<grid, block, 0, st>>>(P, nprob, slot, epoch, clk);
    SCS_HIP(hipGetLastError());
  }
  return SCS_OK;
}

// W <= 16 active workgroups (W xcd_stride <= 128 in the grid) are always resident together on the
// otherwise idle device; an ordinary launch avoids the cooperative queue's extra latency on both
// sides of every epoch, and every wait is bounded.
template <int RPT, int CPT, int WR, bool BF16>
int launch_t(hipStream_t st, InnerArgs& a) {
  dim3 grid((unsigned)(a.W * a.xcd_stride)), block(kInnerThreads);
  inner_epoch_kernel<RPT, CPT, WR, BF16><<<grid, block, 0, st>>>(a);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

// The instantiated layouts: WR = 1 with up to 4 row and 4 column groups per thread (b <= 64,
// 512-column slices); WR = 2 and 4 with up to 2 column groups (128- and 64-column slices) and up to
// 4 row groups (b <= 128 and 256).
struct Layout {
  int rpt, cpt, wr;
};

bool layout_ok(const Layout& L) {
  if (L.rpt != 1 && L.rpt != 2 && L.rpt != 4) return false;
  if (L.wr == 1) return L.cpt >= 1 && L.cpt <= 4;
  if (L.wr == 2 || L.wr == 4) return L.cpt >= 1 && L.cpt <= 2;
  return false;
}

// Rows per thread rounded up to an instantiated count.
int round_rpt(int64_t r) { return r <= 1 ? 1 : r <= 2 ? 2 : r <= 4 ? 4 : 8; }

// Layout for b rows and a slice of `slice` columns: wave_rows > 0 is taken as given; 0 takes the
// fewest wave-rows that hold b rows (64 each), the rule the batched launches use, so that a single
// solve and the same problem inside a batch sum in the same order.
Layout choose_layout(int b, int64_t slice, int wave_rows) {
  int wr = wave_rows;
  if (wr <= 0) {
    wr = 1;
    while (wr < 4 && cdiv(b, wr) > 64) wr *= 2;
  }
  Layout L;
  L.wr = wr;
  L.rpt = round_rpt(cdiv(cdiv(b, wr), 16));
  L.cpt = (int)cdiv(slice, 16 * (8 / (wr > 0 ? wr : 1)));
  return L;
}

template <bool BF16>
int launch_layout(hipStream_t st, InnerArgs& a, const Layout& L) {
#define SCS_INNER_CASE(R, C, WRV) \
  if (L.rpt == R && L.cpt == C && L.wr == WRV) return launch_t<R, C, WRV, BF16>(st, a);
  SCS_INNER_CASE(1, 1, 1) SCS_INNER_CASE(1, 2, 1) SCS_INNER_CASE(1, 3, 1) SCS_INNER_CASE(1, 4, 1)
  SCS_INNER_CASE(2, 1, 1) SCS_INNER_CASE(2, 2, 1) SCS_INNER_CASE(2, 3, 1) SCS_INNER_CASE(2, 4, 1)
  SCS_INNER_CASE(4, 1, 1) SCS_INNER_CASE(4, 2, 1) SCS_INNER_CASE(4, 3, 1) SCS_INNER_CASE(4, 4, 1)
  SCS_INNER_CASE(1, 1, 2) SCS_INNER_CASE(1, 2, 2) SCS_INNER_CASE(2, 1, 2) SCS_INNER_CASE(2, 2, 2)
  SCS_INNER_CASE(4, 1, 2) SCS_INNER_CASE(4, 2, 2)
  SCS_INNER_CASE(1, 1, 4) SCS_INNER_CASE(1, 2, 4) SCS_INNER_CASE(2, 1, 4) SCS_INNER_CASE(2, 2, 4)
  SCS_INNER_CASE(4, 1, 4) SCS_INNER_CASE(4, 2, 4)
#undef SCS_INNER_CASE
  set_error("inner loop: no kernel for this minibatch, slice width and wave-row count");
  return SCS_EINVAL;
}

template <bool BF16>
int launch_layout_batched(hipStream_t st, const BatchProb* P, int nprob, int W, const Layout& L, int slot,
                          int64_t epoch, const int* clk) {
#define SCS_INNER_CASE(R, C, WRV) \
  if (L.rpt == R && L.cpt == C && L.wr == WRV) return launch_bt<R, C, WRV, BF16>(st, P, nprob, W, slot, epoch, clk);
  SCS_INNER_CASE(1, 1, 1) SCS_INNER_CASE(1, 2, 1) SCS_INNER_CASE(1, 3, 1) SCS_INNER_CASE(1, 4, 1)
  SCS_INNER_CASE(2, 1, 1) SCS_INNER_CASE(2, 2, 1) SCS_INNER_CASE(2, 3, 1) SCS_INNER_CASE(2, 4, 1)
  SCS_INNER_CASE(4, 1, 1) SCS_INNER_CASE(4, 2, 1) SCS_INNER_CASE(4, 3, 1) SCS_INNER_CASE(4, 4, 1)
  SCS_INNER_CASE(4, 1, 2) SCS_INNER_CASE(4, 2, 2) SCS_INNER_CASE(4, 1, 4) SCS_INNER_CASE(4, 2, 4)
#undef SCS_INNER_CASE
  set_error("batched inner loop: no kernel for this minibatch and slice width");
  return SCS_EINVAL;
}

}  // namespace

int inner_default_workgroups(int64_t d) {
  // measured on MI355X at d = 1000: 64 columns per workgroup beats 128 (the per-step chain is
  // dominated by latency, so less work per workgroup wins until the exchange cost takes over)
  int64_t W = cdiv(d, 64);
  if (W < 1) W = 1;
  if (W > 16) W = 16;
  return (int)W;
}

int launch_inner_epoch(hipStream_t st, InnerArgs& a, int bf16) {
  if (a.wave_rows == kInnerLookahead) return launch_inner_epoch_lookahead(st, a, bf16);
  if (a.b < 1 || a.b > kInnerMaxB || a.m < 1 || a.W < 1 || a.W > 16) {
    set_error("inner loop: need 1 <= b <= 256, m >= 1, 1 <= workgroups <= 16");
    return SCS_EINVAL;
  }
  if (a.ldx % 4 != 0 || a.ldr != a.ldx) {
    set_error("inner loop: data and regularizer rows need one leading dimension, a multiple of 4");
    return SCS_EINVAL;
  }
  if (a.wave_rows != 0 && a.wave_rows != 1 && a.wave_rows != 2 && a.wave_rows != 4) {
    set_error("inner loop: wave_rows must be 0, 1, 2, 4 or SCS_LOOKAHEAD");
    return SCS_EINVAL;
  }
  a.slice = cdiv(cdiv(a.d, a.W), 4) * 4;
  const Layout L = choose_layout(a.b, a.slice, a.wave_rows);
  if (!layout_ok(L)) {
    set_error("inner loop: slice too wide or minibatch too large for the wave-row count (at most 512 columns "
              "per workgroup with one wave-row, 128 with two, 64 with four; at most 64 rows per wave-row)");
    return SCS_EINVAL;
  }
  return bf16 ? launch_layout<true>(st, a, L) : launch_layout<false>(st, a, L);
}

int inner_layout_wave_rows(int b, int64_t d, int W, int wave_rows) {
  return choose_layout(b, cdiv(cdiv(d, W), 4) * 4, wave_rows).wr;
}

int launch_inner_epoch_batched(hipStream_t st, const BatchProb* P, int nprob, int W, int64_t max_slice, int max_b,
                               int bf16, int epoch_slot, int64_t epoch, const int* clk) {
  if (nprob < 1) return SCS_OK;
  if (max_b < 1 || max_b > kInnerMaxB || W < 1 || W > 16) {
    set_error("batched inner loop: need 1 <= b <= 256 and 1 <= workgroups <= 16");
    return SCS_EINVAL;
  }
  // one wave-row up to b = 64 (any slice up to 512 columns); beyond, 64 rows per wave-row
  Layout L;
  L.wr = max_b <= 64 ? 1 : max_b <= 128 ? 2 : 4;
  L.rpt = L.wr == 1 ? round_rpt(cdiv(max_b, 16)) : 4;
  L.cpt = (int)cdiv(max_slice, 16 * (8 / L.wr));
  if (!layout_ok(L)) {
    set_error("batched inner loop: column slice too wide for the minibatch (b > 64 needs slices of at most "
              "128 columns, b > 128 at most 64)");
    return SCS_EINVAL;
  }
  return bf16 ? launch_layout_batched<true>(st, P, nprob, W, L, epoch_slot, epoch, clk)
              : launch_layout_batched<false>(st, P, nprob, W, L, epoch_slot, epoch, clk);
}

}  // namespace scs
