// Random numbers on the device: the Gaussian test matrix of the range finder and the
// importance-sampled component indices of SVRG (Alg. 1, q_i proportional to beta_i).
//
// Index draws use integer arithmetic only: the beta_i are quantized to fixed-point weights,
// prefix-summed in uint64 (exact, order independent) and inverted with a binary search on a
// 64-bit uniform from Philox4x32-10, so the stream is reproducible bit for bit.
#include "scs_internal.h"

namespace scs {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanPerThread = 8;
constexpr int kScanTile = kScanThreads * kScanPerThread;
constexpr int kMaxStatParts = 256;  // partial (max, sum) pairs the scan kernel stages in LDS

// Gaussian element e: Philox call c = e / 4, counter (c_lo, c_hi, 0, 1); two Box-Muller pairs.
__global__ void gaussian_kernel(uint64_t seed, int64_t count, float* out) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c * 4 >= count) return;
  U4 x = philox4x32_10(U4{(uint32_t)c, (uint32_t)((uint64_t)c >> 32), 0u, 1u}, (uint32_t)seed,
                       (uint32_t)(seed >> 32));
  const double inv = 1.0 / 4294967296.0;
  double u0 = ((double)x.x + 0.5) * inv, u1 = ((double)x.y + 0.5) * inv;
  double u2 = ((double)x.z + 0.5) * inv, u3 = ((double)x.w + 0.5) * inv;
  double r01 = sqrt(-2.0 * log(u0)), r23 = sqrt(-2.0 * log(u2));
  const double two_pi = 2.0 * 3.141592653589793;
  double z[4] = {r01 * cos(two_pi * u1), r01 * sin(two_pi * u1), r23 * cos(two_pi * u3), r23 * sin(two_pi * u3)};
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (c * 4 + q < count) out[c * 4 + q] = (float)z[q];
}

// Partial max and sum of beta (FP64) per workgroup; non-finite values poison the max.
template <typename BT>
__global__ void beta_stats_partial(const BT* beta, int64_t N, double* part) {
  double mx = 0.0, sm = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    double b = (double)beta[i];
    if (!(b >= 0.0) || isinf(b)) b = __longlong_as_double(0x7ff8000000000000ll);
    mx = (isnan(mx) || isnan(b)) ? __longlong_as_double(0x7ff8000000000000ll) : fmax(mx, b);
    sm += b;
  }
  __shared__ double smx[16], ssm[16];
  double wm = mx, ws = warp_sum_d(sm);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    double t = __shfl_xor(wm, o);
    wm = (isnan(wm) || isnan(t)) ? __longlong_as_double(0x7ff8000000000000ll) : fmax(wm, t);
  }
  int wid = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (lane == 0) {
    smx[wid] = wm;
    ssm[wid] = ws;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double m2 = 0.0, s2 = 0.0;
    for (int w = 0; w < (int)blockDim.x / 64; ++w) {
      m2 = (isnan(m2) || isnan(smx[w])) ? __longlong_as_double(0x7ff8000000000000ll) : fmax(m2, smx[w]);
      s2 += ssm[w];
    }
    part[2 * blockIdx.x] = m2;
    part[2 * blockIdx.x + 1] = s2;
  }
}

// Quantize to W_i = max(1, rint(beta_i * scale)) (0 for beta_i = 0) and scan one tile (inclusive).
// uniform: every component gets weight 1 (q_i = 1/N) while the sum of beta still goes to the state
template <typename BT>
__global__ void quantize_scan_tile(const BT* beta, int64_t N, const double* part, int nparts, uint64_t* cum,
                                   uint64_t* tile_sum, SolveState* state, int uniform) {
  __shared__ double s_scale;
  __shared__ uint64_t s_warp[kScanThreads / 64];
  __shared__ double s_part[2 * kMaxStatParts];
  // the partials reach LDS in one coalesced pass; the first wave combines them: lane t takes partials
  // t, t + 64, ... in order, then a butterfly over the wave (lane 0's sum is the one kept). The max, and
  // so the scale and every quantized weight, does not depend on the order. (A serial walk by one thread
  // cost about 20 us per launch from LDS, and about 40 us from global memory.)
  for (int e = threadIdx.x; e < 2 * nparts; e += blockDim.x) s_part[e] = part[e];
  __syncthreads();
  if (threadIdx.x < 64) {
    auto nanmax = [](double a, double b) {
      return (isnan(a) || isnan(b)) ? __longlong_as_double(0x7ff8000000000000ll) : fmax(a, b);
    };
    double mx = 0.0, sm = 0.0;
    for (int p = threadIdx.x; p < nparts; p += 64) {
      mx = nanmax(mx, s_part[2 * p]);
      sm += s_part[2 * p + 1];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      mx = nanmax(mx, __shfl_xor(mx, o));
      sm += __shfl_xor(sm, o);
    }
    int lg = 0;
    while (((int64_t)1 << lg) < (N < 2 ? 2 : N)) ++lg;
    double two_b = ldexp(1.0, 62 - lg);
    if (threadIdx.x == 0) {
      s_scale = (mx > 0.0 && !isnan(mx)) ? two_b / mx : 0.0;
      if (blockIdx.x == 0 && state) state->beta_sum = sm;
    }
  }
  __syncthreads();
  const double scale = s_scale;
  int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPerThread;
  uint64_t v[kScanPerThread];
  uint64_t run = 0;
#pragma unroll
  for (int q = 0; q < kScanPerThread; ++q) {
    int64_t i = base + q;
    uint64_t wq = 0;
    if (i < N) {
      double b = (double)beta[i];
      if (uniform) {
        wq = 1ull;
      } else if (b > 0.0) {
        double r = rint(b * scale);
        wq = r < 1.0 ? 1ull : (uint64_t)r;
      }
    }
    run += wq;
    v[q] = run;
  }
  // exclusive scan of the per-thread totals across the workgroup
  uint64_t tot = run, incl = tot;
  int lane = threadIdx.x % 64, wid = threadIdx.x / 64;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint64_t t = __shfl_up(incl, o);
    if (lane >= o) incl += t;
  }
  if (lane == 63) s_warp[wid] = incl;
  __syncthreads();
  uint64_t off = 0;
  for (int w = 0; w < wid; ++w) off += s_warp[w];
  uint64_t excl = off + incl - tot;
#pragma unroll
  for (int q = 0; q < kScanPerThread; ++q) {
    int64_t i = base + q;
    if (i < N) cum[i] = v[q] + excl;
  }
  if (threadIdx.x == kScanThreads - 1) tile_sum[blockIdx.x] = excl + tot;
}

// Exclusive scan of the tile totals (single workgroup, sequential over chunks of 256).
__global__ void scan_tile_sums(uint64_t* tile_sum, int64_t ntiles) {
  __shared__ uint64_t s_warp[4];
  __shared__ uint64_t s_carry;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (int64_t c0 = 0; c0 < ntiles; c0 += 256) {
    int64_t i = c0 + threadIdx.x;
    uint64_t x = i < ntiles ? tile_sum[i] : 0, incl = x;
    int lane = threadIdx.x % 64, wid = threadIdx.x / 64;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      uint64_t t = __shfl_up(incl, o);
      if (lane >= o) incl += t;
    }
    if (lane == 63) s_warp[wid] = incl;
    __syncthreads();
    uint64_t off = s_carry;
    for (int w = 0; w < wid; ++w) off += s_warp[w];
    if (i < ntiles) tile_sum[i] = off + incl - x;
    __syncthreads();
    if (threadIdx.x == 255) s_carry = off + incl;
    __syncthreads();
  }
}

__global__ void add_tile_offsets(uint64_t* cum, int64_t N, const uint64_t* tile_off, SolveState* state) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) cum[i] += tile_off[i / kScanTile];
  if (i == N - 1 && state) state->wsum = (double)(cum[i]);
}

__device__ __forceinline__ int64_t upper_bound_u64(const uint64_t* cum, int64_t N, uint64_t u) {
  int64_t lo = 0, hi = N;  // first index with cum > u
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (cum[mid] > u) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

// 1 / (n q_i) with q_i = W_i / T, in FP64, then rounded to the scale's type.
template <typename ST>
__device__ __forceinline__ ST inv_nq(const uint64_t* cum, int64_t i, int64_t n_rows, uint64_t T) {
  uint64_t wi = cum[i] - (i > 0 ? cum[i - 1] : 0ull);
  return (ST)((double)T / ((double)n_rows * (double)wi));
}

// Draws `count` indices for consecutive epochs epoch0, epoch0 + 1, ... (per_epoch draws each); draw
// g of epoch e uses Philox call g/2 with counter (call_lo, call_hi, e, 0), words (x0, x1) for even g
// and (x2, x3) for odd g, so a multi-epoch launch draws exactly what per-epoch launches would.
template <typename ST>
__device__ __forceinline__ void sample_one(const uint64_t* cum, int64_t N, int64_t n_rows, uint64_t seed,
                                           uint32_t epoch0, int64_t per_epoch, int64_t g, int32_t* idx,
                                           ST* scale);

template <typename ST>
__global__ void sample_kernel(const uint64_t* cum, int64_t N, int64_t n_rows, uint64_t seed, uint32_t epoch0,
                              int64_t per_epoch, int64_t count, int32_t* idx, ST* scale,
                              const SolveState* state) {
  if (state && state->done) return;
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= count) return;
  sample_one(cum, N, n_rows, seed, epoch0, per_epoch, g, idx, scale);
}

// Batched: draw g of the launch belongs to problem p with draw_prefix[p] <= g < draw_prefix[p+1];
// each problem draws `groups` epochs of its own m b draws from its own weights (same stream as a
// single solve with the same seed).
__global__ void sample_batched_kernel(const BatchProb* P, int nprob, const int64_t* draw_prefix, int64_t total,
                                      uint64_t seed, uint32_t epoch0, const int* clk) {
  if (clk) {  // epochs replayed from a graph: draw a group of epochs when the device's epoch starts one
    if (clk[0] >= clk[1] || clk[0] % kEpochGroup != 0) return;
    epoch0 = (uint32_t)clk[0];
  }
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int p = find_prob(draw_prefix, nprob, g);
  const BatchProb& q = P[p];
  if (q.state->done) return;
  sample_one<float>(q.cum, q.N, q.n, seed, epoch0, q.draws, g - draw_prefix[p], q.idx, q.scale);
}

template <typename ST>
__device__ __forceinline__ void sample_one(const uint64_t* cum, int64_t N, int64_t n_rows, uint64_t seed,
                                           uint32_t epoch0, int64_t per_epoch, int64_t g, int32_t* idx,
                                           ST* scale) {
  const uint32_t epoch = epoch0 + (uint32_t)(g / per_epoch);
  const int64_t gl = g % per_epoch;
  uint64_t c = (uint64_t)gl >> 1;
  U4 x = philox4x32_10(U4{(uint32_t)c, (uint32_t)(c >> 32), epoch, 0u}, (uint32_t)seed, (uint32_t)(seed >> 32));
  uint64_t r = (gl & 1) ? (((uint64_t)x.z << 32) | x.w) : (((uint64_t)x.x << 32) | x.y);
  uint64_t T = cum[N - 1];
  uint64_t u = __umul64hi(r, T);
  int64_t i = upper_bound_u64(cum, N, u);
  if (i >= N) i = N - 1;  // unreachable for u < T; kept as a guard
  idx[g] = (int32_t)i;
  if (scale) scale[g] = inv_nq<ST>(cum, i, n_rows, T);
}

template <typename ST>
__global__ void index_scale_kernel(const uint64_t* cum, int64_t N, int64_t n_rows, const int32_t* idx,
                                   int64_t count, ST* scale, const SolveState* state) {
  if (state && state->done) return;
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= count) return;
  int64_t i = idx[g];
  if (i < 0) i = 0;
  if (i >= N) i = N - 1;
  scale[g] = inv_nq<ST>(cum, i, n_rows, cum[N - 1]);
}

constexpr int kStatBlocks = 256;
static_assert(kStatBlocks <= kMaxStatParts, "the scan kernel stages at most kMaxStatParts partials");

}  // namespace

int launch_gaussian(hipStream_t st, uint64_t seed, int64_t count, float* out) {
  if (count <= 0) return SCS_OK;
  int64_t calls = cdiv(count, 4);
  gaussian_kernel<<<dim3((unsigned)cdiv(calls, 256)), dim3(256), 0, st>>>(seed, count, out);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

// scratch layout (in doubles): [2*kStatBlocks partials][tile sums as uint64]
int64_t sampler_scratch_len(int64_t N) { return 2 * kStatBlocks + cdiv(N, kScanTile) + 1; }

template <typename BT>
static int sampler_prepare(hipStream_t st, const BT* beta, int64_t N, uint64_t* cum, double* scratch,
                           int64_t scratch_len, SolveState* state, int uniform) {
  if (N <= 0) return SCS_EINVAL;
  if (scratch_len < sampler_scratch_len(N)) return SCS_EINVAL;
  double* part = scratch;
  uint64_t* tiles = reinterpret_cast<uint64_t*>(scratch + 2 * kStatBlocks);
  int64_t ntiles = cdiv(N, kScanTile);
  beta_stats_partial<BT><<<kStatBlocks, 256, 0, st>>>(beta, N, part);
  SCS_HIP(hipGetLastError());
  quantize_scan_tile<BT><<<dim3((unsigned)ntiles), dim3(kScanThreads), 0, st>>>(beta, N, part, kStatBlocks, cum,
                                                                                tiles, state, uniform);
  SCS_HIP(hipGetLastError());
  scan_tile_sums<<<1, 256, 0, st>>>(tiles, ntiles);
  SCS_HIP(hipGetLastError());
  add_tile_offsets<<<dim3((unsigned)cdiv(N, 256)), dim3(256), 0, st>>>(cum, N, tiles, state);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_sampler_prepare(hipStream_t st, const float* beta, int64_t N, uint64_t* cum, double* scratch,
                           int64_t scratch_len, SolveState* state, int uniform) {
  return sampler_prepare(st, beta, N, cum, scratch, scratch_len, state, uniform);
}

int launch_sampler_prepare(hipStream_t st, const double* beta, int64_t N, uint64_t* cum, double* scratch,
                           int64_t scratch_len, SolveState* state, int uniform) {
  return sampler_prepare(st, beta, N, cum, scratch, scratch_len, state, uniform);
}

template <typename ST>
static int sample(hipStream_t st, const uint64_t* cum, int64_t N, int64_t n_rows, uint64_t seed, int epoch,
                  int64_t per_epoch, int64_t count, int32_t* idx, ST* scale, const SolveState* state) {
  if (count <= 0) return SCS_OK;
  if (per_epoch <= 0) per_epoch = count;
  sample_kernel<ST><<<dim3((unsigned)cdiv(count, 256)), dim3(256), 0, st>>>(cum, N, n_rows, seed, (uint32_t)epoch,
                                                                        per_epoch, count, idx, scale, state);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_sample_batched(hipStream_t st, const BatchProb* P, int nprob, const int64_t* draw_prefix,
                          int64_t total_draws, uint64_t seed, int epoch, int groups, const int* clk) {
  (void)groups;
  if (total_draws <= 0) return SCS_OK;
  sample_batched_kernel<<<dim3((unsigned)cdiv(total_draws, 256)), dim3(256), 0, st>>>(P, nprob, draw_prefix,
                                                                                       total_draws, seed,
                                                                                       (uint32_t)epoch, clk);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_sample(hipStream_t st, const uint64_t* cum, int64_t N, int64_t n_rows, uint64_t seed, int epoch,
                  int64_t per_epoch, int64_t count, int32_t* idx, float* scale, const SolveState* state) {
  return sample(st, cum, N, n_rows, seed, epoch, per_epoch, count, idx, scale, state);
}

int launch_sample(hipStream_t st, const uint64_t* cum, int64_t N, int64_t n_rows, uint64_t seed, int epoch,
                  int64_t per_epoch, int64_t count, int32_t* idx, double* scale, const SolveState* state) {
  return sample(st, cum, N, n_rows, seed, epoch, per_epoch, count, idx, scale, state);
}

template <typename ST>
static int index_scale(hipStream_t st, const uint64_t* cum, int64_t N, int64_t n_rows, const int32_t* idx,
                       int64_t count, ST* scale, const SolveState* state) {
  if (count <= 0) return SCS_OK;
  index_scale_kernel<ST><<<dim3((unsigned)cdiv(count, 256)), dim3(256), 0, st>>>(cum, N, n_rows, idx, count,
                                                                                 scale, state);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_index_scale(hipStream_t st, const uint64_t* cum, int64_t N, int64_t n_rows, const int32_t* idx,
                       int64_t count, float* scale, const SolveState* state) {
  return index_scale(st, cum, N, n_rows, idx, count, scale, state);
}

int launch_index_scale(hipStream_t st, const uint64_t* cum, int64_t N, int64_t n_rows, const int32_t* idx,
                       int64_t count, double* scale, const SolveState* state) {
  return index_scale(st, cum, N, n_rows, idx, count, scale, state);
}

}  // namespace scs
