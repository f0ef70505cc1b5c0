// C-ABI of libscs: context, workspace and the orchestration of Sketched Preconditioned SVRG
// (Alg. 3): sketch -> preconditioner -> SVRG epochs (full-gradient pass + persistent inner loop)
// -> w = P^{-1/2} w~. Every arithmetic step runs in the HIP kernels of this library; the host
// only validates arguments, sizes scratch buffers, enqueues launches and reads status records.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "scs_internal.h"

using namespace scs;

namespace {
thread_local std::string g_last_error;
}

void scs::set_error(const std::string& msg) { g_last_error = msg; }

struct scs_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  struct Buf {
    void* p = nullptr;
    size_t bytes = 0;
  };
  std::map<std::string, Buf> bufs;
  std::vector<void*> retired;       // buffers replaced by larger ones, freed at the next call's entry
  std::vector<hipEvent_t> events;   // synchronizing events (host waits on them)
  std::vector<hipEvent_t> tevents;  // timing-only events (no system-scope fence when recorded)
  std::map<std::string, std::pair<int, int>> tuned_w;  // autotuned inner-loop (workgroups, wave-rows) per (d, b, precision)
  hipEvent_t tune_ev[2] = {nullptr, nullptr};
  std::vector<hipStream_t> side;       // extra streams for independent per-problem setup work
  std::vector<hipEvent_t> side_events;
  int* stop_flags = nullptr;  // host-pinned, one per epoch: set by the device when the solve is finished
  size_t stop_cap = 0;
  int xcd_stride = 8;
  hipEvent_t fork_ev[2] = {nullptr, nullptr};  // work forked onto side stream 0 inside a single solve, and joined
  hipEvent_t join_ev[2] = {nullptr, nullptr};
};

namespace {

// Scratch buffer `name` with at least `bytes` (contents undefined after growth). A buffer that grows
// is replaced, not freed: work already queued on any of the context's streams may still use it, and
// freeing it here would need a device-wide wait in the middle of enqueueing (the batched setup grows
// its per-lane buffers as it meets wider problems, and such waits serialized its streams). Replaced
// buffers are freed by free_retired at the entry of the next call.
void* wsb(scs_ctx* c, const std::string& name, size_t bytes) {
  if (bytes == 0) bytes = 16;
  auto& b = c->bufs[name];
  if (b.bytes >= bytes) return b.p;
  if (b.p) {
    c->retired.push_back(b.p);
    b.p = nullptr;
    b.bytes = 0;
  }
  size_t want = ((bytes + 4095) / 4096) * 4096;
  if (hipMalloc(&b.p, want) != hipSuccess) {
    set_error("hipMalloc failed for scratch buffer " + name + " (" + std::to_string(want) + " bytes)");
    b.p = nullptr;
    return nullptr;
  }
  b.bytes = want;
  return b.p;
}

// Frees the buffers wsb replaced, after waiting for the device (they may be in use by work of an
// earlier, asynchronous call). Called at the entry of the calls that allocate workspace.
void free_retired(scs_ctx* c) {
  if (c->retired.empty()) return;
  hipDeviceSynchronize();
  for (void* p : c->retired) hipFree(p);
  c->retired.clear();
}

template <class T>
T* ws(scs_ctx* c, const std::string& name, size_t count) {
  return reinterpret_cast<T*>(wsb(c, name, count * sizeof(T)));
}

#define WS(var, T, name, count)                  \
  T* var = ws<T>(ctx, name, (size_t)(count));    \
  if (!var) return SCS_ENOMEM;

// events: the per-epoch decision points the host waits on before it reads that epoch's stop flag.
// They carry no system-scope fence (a fence would write back L2 before every inner loop): the flag
// is a system-scope store of its own, and a stale read only lets the host queue a few more epochs,
// which return at once on the device's done flag. tevents: timing only, also without the fence.
int ensure_events(scs_ctx* c, size_t count, size_t tcount = 0) {
  while (c->events.size() < count) {
    hipEvent_t e;
    SCS_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence | hipEventDisableTiming));
    c->events.push_back(e);
  }
  while (c->tevents.size() < tcount) {
    hipEvent_t e;
    SCS_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    c->tevents.push_back(e);
  }
  return SCS_OK;
}

// count streams besides the context's own (default priority, non-blocking), each with an event
int ensure_side_streams(scs_ctx* c, int count) {
  while ((int)c->side.size() < count) {
    hipStream_t q;
    hipEvent_t e;
    SCS_HIP(hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
    SCS_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    c->side.push_back(q);
    c->side_events.push_back(e);
  }
  return SCS_OK;
}

// Host-pinned (coherent) flags the gradient finalizer writes; the host reads them to stop enqueuing.
int ensure_stop_flags(scs_ctx* c, size_t count) {
  if (c->stop_cap >= count) return SCS_OK;
  if (c->stop_flags) {
    hipStreamSynchronize(c->stream);
    hipHostFree(c->stop_flags);
    c->stop_flags = nullptr;
    c->stop_cap = 0;
  }
  SCS_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->stop_flags), count * sizeof(int), hipHostMallocCoherent));
  c->stop_cap = count;
  return SCS_OK;
}

// Waits until the gradient finish of snapshot q has written its host flag (1: the solve is finished,
// 2: continue), which it writes in every case once it has run. Between reads of the flag the stream is
// queried now and then: an error ends the wait, and so does a drained stream whose flag is still unset.
int wait_stop_flag(scs_ctx* c, hipStream_t st, int q, int* flag) {
  for (uint32_t spin = 1;; ++spin) {
    *flag = __atomic_load_n(c->stop_flags + q, __ATOMIC_ACQUIRE);
    if (*flag) return SCS_OK;
    if ((spin & 255u) == 0) {
      const hipError_t e = hipStreamQuery(st);
      if (e == hipSuccess) {
        *flag = __atomic_load_n(c->stop_flags + q, __ATOMIC_ACQUIRE);
        if (*flag) return SCS_OK;
        set_error("solve: the stream drained without writing the snapshot's stop flag");
        return SCS_EDEVICE;
      }
      if (e != hipErrorNotReady) SCS_HIP(e);
    }
  }
}

struct Guard {  // makes the context's device current for the duration of a call
  int prev = -1;
  explicit Guard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    hipSetDevice(dev);
  }
  ~Guard() {
    if (prev >= 0) hipSetDevice(prev);
  }
};

// m of Alg. 1: the literal step count, else epoch_factor n / b, else 2 n / b
int64_t epoch_steps(const scs_opts& o, int64_t n, int b) {
  if (o.steps > 0) return o.steps;
  if (o.epoch_factor > 0.0) return std::max<int64_t>(1, (int64_t)std::ceil(o.epoch_factor * (double)n / b));
  return cdiv(2 * n, b);
}

// Widest column slice the batched inner loop takes for minibatch b (one wave-row up to b = 64,
// two up to 128, four beyond).
int64_t batched_max_slice(int b) { return b <= 64 ? 512 : b <= 128 ? 128 : 64; }

int choose_workgroups(const scs_opts& o, int64_t d) {
  if (o.workgroups > 0) return o.workgroups;
  // at least enough workgroups for the widest slice the minibatch's layout takes
  return (int)std::min<int64_t>(16, std::max<int64_t>(inner_default_workgroups(d), cdiv(d, batched_max_slice(o.batch))));
}

// Measured choice of the inner loop's launch shape: the workgroup count W (the width of each
// workgroup's column slice) and the wave-row count (how the workgroup's waves split the minibatch's
// rows). A few dozen steps of the epoch kernel run on the problem's own rows, with a scratch
// snapshot, state and exchange buffer, for each candidate; the fastest is kept in the context per
// (d, b, precision).
int autotune_workgroups(scs_ctx* ctx, hipStream_t st, const InnerArgs& base, int bf16, const uint64_t* cum,
                        int64_t N, uint64_t seed, int* W_out, int* wr_out) {
  const std::string key = std::to_string(base.d) + "/" + std::to_string(base.b) + "/" + std::to_string(bf16);
  auto it = ctx->tuned_w.find(key);
  if (it != ctx->tuned_w.end()) {
    *W_out = it->second.first;
    *wr_out = it->second.second;
    return SCS_OK;
  }
  // a layout with wr wave-rows takes at most 64 rows per wave-row and slices of at most 512 (wr = 1),
  // 128 (wr = 2) or 64 (wr = 4) columns; the look-ahead loop b <= 64 and slices of at most 64 columns
  std::vector<std::pair<int, int>> cand;
  for (int cols : {128, 64, 32}) {
    const int W = (int)std::max<int64_t>(1, std::min<int64_t>(16, cdiv(base.d, cols)));
    const int64_t slice = cdiv(cdiv(base.d, W), 4) * 4;
    for (int wr : {1, 2, 4, kInnerLookahead}) {
      if (wr == kInnerLookahead) {
        if (!inner_lookahead_fits(base.b, base.d, W)) continue;
      } else {
        const int64_t max_slice = wr == 1 ? 512 : wr == 2 ? 128 : 64;
        if (cdiv(base.b, wr) > 64 || slice > max_slice) continue;
      }
      const std::pair<int, int> c{W, wr};
      if (std::find(cand.begin(), cand.end(), c) == cand.end()) cand.push_back(c);
    }
  }
  if (cand.empty()) {
    *W_out = inner_default_workgroups(base.d);
    *wr_out = 0;
    return SCS_OK;
  }
  if (cand.size() == 1) {
    *W_out = cand[0].first;
    *wr_out = cand[0].second;
    ctx->tuned_w[key] = cand[0];
    return SCS_OK;
  }
  for (auto& e : ctx->tune_ev)
    if (!e) SCS_HIP(hipEventCreate(&e));
  // every timed run gathers its own rows (a fresh index stream), as a real epoch does: rows already
  // in the caches would favour fewer, wider workgroups
  const int64_t mp = std::min<int64_t>(base.m, 48);
  const int reps = 2, runs = (int)cand.size() * reps;
  WS(twt, float, "at_wt", base.d);
  WS(tmu, float, "at_mu", base.d);
  WS(tidx, int32_t, "at_idx", runs * mp * base.b);
  WS(tsc, float, "at_scale", runs * mp * base.b);
  WS(tstate, SolveState, "at_state", 1);
  WS(txb, uint64_t, "at_xbuf", inner_xbuf_words(16));
  SCS_HIP(hipMemsetAsync(tmu, 0, sizeof(float) * base.d, st));
  SCS_CHECK(launch_sample(st, cum, N, base.n, seed, 0x7fff0000, mp * base.b, runs * mp * base.b, tidx, tsc, nullptr));
  std::pair<int, int> best = cand[0];
  int run = 0;
  float best_ms = 1e30f;
  for (const auto& c : cand) {
    for (int rep = 0; rep < reps; ++rep, ++run) {
      SCS_HIP(hipMemsetAsync(twt, 0, sizeof(float) * base.d, st));
      SCS_HIP(hipMemsetAsync(txb, 0, sizeof(uint64_t) * inner_xbuf_words(16), st));
      SCS_HIP(hipMemcpyAsync(tstate, base.state, sizeof(SolveState), hipMemcpyDeviceToDevice, st));
      InnerArgs a = base;
      a.W = c.first;
      a.wave_rows = c.second;
      a.xcd_stride = c.first > 1 ? ctx->xcd_stride : 1;
      a.m = mp;
      a.idx = tidx + (int64_t)run * mp * base.b;
      a.scale = tsc + (int64_t)run * mp * base.b;
      a.mu = tmu;
      a.wt = twt;
      a.wt_prev = nullptr;
      a.xbuf = txb;
      a.state = tstate;
      a.step_base = 0;
      SCS_HIP(hipEventRecord(ctx->tune_ev[0], st));
      SCS_CHECK(launch_inner_epoch(st, a, bf16));
      SCS_HIP(hipEventRecord(ctx->tune_ev[1], st));
      SCS_HIP(hipEventSynchronize(ctx->tune_ev[1]));
      float ms = 0.f;
      SCS_HIP(hipEventElapsedTime(&ms, ctx->tune_ev[0], ctx->tune_ev[1]));
      if (ms < best_ms) {
        best_ms = ms;
        best = c;
      }
    }
  }
  ctx->tuned_w[key] = best;
  *W_out = best.first;
  *wr_out = best.second;
  return SCS_OK;
}

// Columns of the sketch's Krylov basis, q (k + p), within what the one-workgroup FP64 eigensolver and
// CholeskyQR2 take (136) and within the rank X can have.
bool sketch_width_ok(const scs_opts& o, int k, int64_t n, int64_t d) {
  if (o.krylov_blocks < 0 || o.krylov_blocks > 32) return false;
  const int64_t L = (int64_t)(k + o.oversample) * std::max(1, o.krylov_blocks);
  return L <= d && L <= n && L <= 136;
}

// Device epoch clock of batched and path solves (two ints, see launch_clock_set).
int* ctx_clock(scs_ctx* c) { return ws<int>(c, "epoch_clock", 2); }

// Epochs of a batched or path solve from a captured graph: kEpochGroup epochs whose kernels read the
// epoch number from the device clock are captured once and the graph is replayed, S / kEpochGroup
// times at most; the host checks the stop flags of a replay's epochs while the next replay runs (the
// kernels of finished problems return at once, as in the enqueued mode). On return *s_next is the
// first epoch still to be enqueued by the caller (the remainder, and the final evaluation at epoch S)
// and *stopped says whether every problem already met the stop rule. The stream runs only these
// kernels, so the graph is recorded without memset or event nodes.
template <class F>
int run_epoch_graph(scs_ctx* ctx, hipStream_t st, int S, F& epoch_launches, int* s_next, bool* stopped) {
  *s_next = 0;
  *stopped = false;
  const int E = kEpochGroup, R = S / E;
  if (R < 1) return SCS_OK;
  int* clk = ctx_clock(ctx);
  if (!clk) return SCS_ENOMEM;
  SCS_CHECK(launch_clock_set(st, clk, 0, S));
  SCS_CHECK(ensure_events(ctx, 0, (size_t)4 + R));
  // captured on the context's side stream (the caller's stream may be the null stream, which cannot
  // be captured); the graph is launched on the caller's stream
  SCS_CHECK(ensure_side_streams(ctx, 1));
  hipStream_t cs = ctx->side[0];
  hipGraph_t g = nullptr;
  SCS_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  int rc = SCS_OK;
  for (int e = 0; e < E && rc >= 0; ++e) rc = epoch_launches(cs, -1, clk);
  const hipError_t ec = hipStreamEndCapture(cs, &g);
  if (rc < 0) {
    if (g) hipGraphDestroy(g);
    return rc;
  }
  SCS_HIP(ec);
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  SCS_HIP(ei);
  hipEvent_t* tev = ctx->tevents.data();
  int r = 0;
  for (; r < R; ++r) {
    const hipError_t el = hipGraphLaunch(exec, st);
    if (el != hipSuccess) {
      hipStreamSynchronize(st);
      hipGraphExecDestroy(exec);
      SCS_HIP(el);
    }
    SCS_HIP(hipEventRecord(tev[4 + r], st));
    if (r >= 1) {
      SCS_HIP(hipEventSynchronize(tev[4 + r - 1]));
      for (int e = (r - 1) * E; e < r * E; ++e)
        if (__atomic_load_n(ctx->stop_flags + e, __ATOMIC_ACQUIRE)) *stopped = true;
      if (*stopped) {
        ++r;
        break;
      }
    }
  }
  SCS_HIP(hipStreamSynchronize(st));
  hipGraphExecDestroy(exec);
  for (int e = (r - 1) * E; e < r * E && !*stopped; ++e)
    if (__atomic_load_n(ctx->stop_flags + e, __ATOMIC_ACQUIRE)) *stopped = true;
  *s_next = r * E;
  return SCS_OK;
}

// Sketch of Alg. 2 with one block. Fills ws buffers "U32" (d x k), "UT32" (k x d), "U64", "lam",
// and, if want_z, "Z" = X U~ (n x k, leading dimension gemm_wide_kpad(k), zero up to the next multiple
// of 16) computed as (X Q) V_k. rank_def set if CholeskyQR broke down.
// flags_out (device, 2 ints, nullable): where CholeskyQR's breakdown flags go; when given, the call
// does not wait for them and *rank_def is left unchanged (the caller reads the flags later).
// st_in / sfx: the stream to use and a suffix for the names of its workspace buffers (so that
// sketches of different problems can run on different streams at once).
// CholeskyQR2 of Yb (d x l, FP64): Qout = Yb R1^{-1} R2^{-1} (leading dimension ldq), QTout (nullable)
// = Qout^T in FP32; f[0], f[1] receive the two factorizations' breakdown flags. G, Rinv: l x l, Q1: d x l,
// Rp: l (l + 1) / 2 + l, Gp: gram64_parts(d) l^2.
// gate (device int, nullable): with it, the second pass takes the symmetric orthogonalization
// Q = Q1 (I + E)^{-1/2} by its binomial series (first order up to l max|E_ij| = 1e-7, second order
// up to 1e-5) when Q1^T Q1 = I + E is that close to I (the usual case: the first pass leaves E of order
// kappa(Y)^2 u), and the Cholesky pass otherwise.
int cholqr2_64(hipStream_t st, int64_t d, int l, const double* Yb, double* Qout, int64_t ldq, float* QTout, int* f,
               double* G, double* Rinv, double* Q1, double* Rp, double* Gp, int* gate) {
  SCS_CHECK(launch_gram64(st, Yb, d, l, Gp, G));
  SCS_CHECK(launch_chol_inv64(st, G, 1, l, Rp, Rinv, f));
  SCS_CHECK(launch_gemm64(st, d, l, l, Yb, l, 1, Rinv, l, 1, Q1, l, nullptr, 0));
  SCS_CHECK(launch_gram64(st, Q1, d, l, Gp, G));
  if (gate) SCS_CHECK(launch_lowdin64(st, G, l, Rinv, f + 1, gate));
  SCS_CHECK(launch_chol_inv64(st, G, 1, l, Rp, Rinv, f + 1, gate));
  SCS_CHECK(launch_gemm64(st, d, l, l, Q1, l, 1, Rinv, l, 1, Qout, ldq, nullptr, 0));
  if (QTout) SCS_CHECK(launch_gemm64(st, l, d, l, Rinv, 1, l, Q1, 1, l, nullptr, 0, QTout, d));  // R2^{-T} Q1^T
  return SCS_OK;
}

// A sketch in parts, for the batched setup (buffers that cross parts are named with the caller's
// persistent suffix). stage 0: up to the Rayleigh-Ritz matrix B (L x L), with the basis Q (d x L) and
// Wq = X Q (n x Lp), for a batched eigensolver and lift; 1: the range finder alone, up to Y (d x l),
// for a batched CholeskyQR2 that writes Q64 and QT32 of the same suffix (one Krylov block); 2: from
// that Q up to B, as stage 0.
struct SketchSplit {
  int stage = 0;
  double* Y = nullptr;
  int l = 0;
  const double* B = nullptr;
  const double* Q = nullptr;
  int L = 0;
  const float* Wq = nullptr;
  int64_t Lp = 0;
};

int sketch_impl(scs_ctx* ctx, const float* X, int64_t n, int64_t d, int64_t ldx, int k, const scs_opts& o,
                bool want_z, bool* rank_def, int* flags_out = nullptr, hipStream_t st_in = nullptr,
                const std::string& sfx = "", hipEvent_t x_done = nullptr, SketchSplit* split = nullptr,
                const std::string& psfx = "") {
  hipStream_t st = st_in ? st_in : ctx->stream;
  const std::string& ksfx = split ? psfx : sfx;  // buffers that must outlive the call in split mode
  const int stage = split ? split->stage : 0;
  const int l = k + o.oversample;
  // Rayleigh-Ritz (X Q, its Gram, Z = X U~) follows the precision; the range finder (X Omega, X^T T and
  // the further Krylov blocks) reads X in BF16 (FP32 accumulation) unless FP32 is asked for: it only
  // fixes the subspace that Rayleigh-Ritz then resolves
  const int bf = o.precision == SCS_PREC_MIXED;
  const int bf_range = bf || !o.sketch_fp32;
  // T = X Omega (n x l, leading dimension l rounded up to 16 and zero-filled), then Y = X^T T (d x l),
  // split over row chunks, summed in FP64
  const int64_t lp = cdiv(l, 16) * 16;
  WS(T, float, std::string("T") + sfx, (size_t)n * lp);
  int64_t nchunks = gemm_tn_splitk_chunks(n, d, l, X, ldx, T, lp);
  int64_t chunk = cdiv(n, nchunks);
  nchunks = cdiv(n, chunk);
  WS(part, float, std::string("partial") + sfx, (size_t)nchunks * d * l);
  WS(Y, double, std::string("Y64") + ksfx, (size_t)d * l);
  if (stage != 2) {
    // Omega^T (l x d)
    const float* OmT = o.omega;
    if (!OmT) {
      WS(om, float, std::string("omega") + sfx, (size_t)l * d);
      SCS_CHECK(launch_gaussian(st, o.seed, (int64_t)l * d, om));
      OmT = om;
    }
    SCS_CHECK(launch_gemm_nt_longk(st, bf_range, X, n, d, ldx, OmT, l, d, T, lp, true));
    SCS_CHECK(launch_gemm_tn_splitk(st, bf_range, X, n, d, ldx, T, l, lp, part, chunk, nchunks));
    SCS_CHECK(launch_reduce_partials_f64(st, part, nchunks, d * l, 1.0, Y));
    if (stage == 1) {
      split->Y = Y;
      split->l = l;
      return SCS_OK;
    }
  }
  // CholeskyQR2: Q1 = Y R1^{-1}, Q = Q1 R2^{-1}
  WS(Rinv, double, std::string("Rinv64") + sfx, (size_t)l * l);
  WS(Q1, double, std::string("Q1_64") + sfx, (size_t)d * l);
  WS(Q, double, std::string("Q64") + ksfx, (size_t)d * l);
  WS(QT32, float, std::string("QT32") + ksfx, (size_t)l * d);
  int* flags = flags_out;
  if (!flags) {
    flags = ws<int>(ctx, "cholflags" + sfx, 2);
    if (!flags) return SCS_ENOMEM;
  }
  const int q = std::max(1, o.krylov_blocks);
  int* bflags = flags;  // with several blocks, each block's CholeskyQR2 flags, ORed into flags at the end
  if (q > 1) {
    bflags = ws<int>(ctx, "blockflags" + sfx, (size_t)2 * q);
    if (!bflags) return SCS_ENOMEM;
  }
  WS(G, double, std::string("G64") + sfx, (size_t)l * l);
  WS(Rp, double, std::string("Rp64") + sfx, (size_t)l * (l + 1) / 2 + l);
  WS(Gp, double, std::string("Gpart64") + sfx, (size_t)gram64_parts(d) * l * l);
  WS(cgate, int, std::string("chol_gate") + sfx, 1);
  auto cholqr2 = [&](const double* Yb, double* Qout, int64_t ldq, float* QTout, int* f) -> int {
    return cholqr2_64(st, d, l, Yb, Qout, ldq, QTout, f, G, Rinv, Q1, Rp, Gp, cgate);
  };
  int L = l;            // columns of the orthonormal basis handed to Rayleigh-Ritz
  const double* Qb = Q; // that basis, d x L (leading dimension L)
  if (q == 1) {
    if (stage != 2) SCS_CHECK(cholqr2(Y, Q, l, QT32, flags));
  } else {
    // Block Lanczos (Alg. 2): the Krylov space [C Omega, C^2 Omega, ..., C^q Omega] (C = X^T X / n, up to
    // the scale of each block), built block by block: block j is C applied to the orthonormal block j-1,
    // projected twice against the blocks before it (block Gram-Schmidt) and orthonormalized by CholeskyQR2.
    // Its span is the span of the stacked Krylov blocks.
    L = q * l;
    WS(Qall, double, std::string("Qall64") + ksfx, (size_t)d * L);
    WS(QTb, float, std::string("QTb32") + sfx, (size_t)l * d);
    WS(Yj, double, std::string("Yj64") + sfx, (size_t)d * l);
    WS(Zj, double, std::string("Zj64") + sfx, (size_t)L * l);
    WS(Wj, double, std::string("Wj64") + sfx, (size_t)d * l);
    SCS_CHECK(cholqr2(Y, Qall, L, QTb, bflags));
    for (int j = 1; j < q; ++j) {
      // Yj = X^T (X Q_{j-1}) / n
      SCS_CHECK(launch_gemm_nt_longk(st, bf_range, X, n, d, ldx, QTb, l, d, T, lp, true));
      SCS_CHECK(launch_gemm_tn_splitk(st, bf_range, X, n, d, ldx, T, l, lp, part, chunk, nchunks));
      SCS_CHECK(launch_reduce_partials_f64(st, part, nchunks, d * l, 1.0 / (double)n, Yj));
      const int64_t Pc = (int64_t)j * l;  // columns of the blocks before j
      for (int pass = 0; pass < 2; ++pass) {
        SCS_CHECK(launch_gemm64(st, Pc, l, d, Qall, 1, L, Yj, l, 1, Zj, l, nullptr, 0));   // Z = Q_prev^T Yj
        SCS_CHECK(launch_gemm64(st, d, l, Pc, Qall, L, 1, Zj, l, 1, Wj, l, nullptr, 0));   // W = Q_prev Z
        SCS_CHECK(launch_axpy64(st, (int64_t)d * l, -1.0, Wj, Yj));
      }
      SCS_CHECK(cholqr2(Yj, Qall + Pc, L, j + 1 < q ? QTb : nullptr, bflags + 2 * j));
    }
    SCS_CHECK(launch_or_flags(st, bflags, 2 * q, flags));
    WS(QTall, float, std::string("QTall32") + sfx, (size_t)L * d);
    SCS_CHECK(launch_transpose64to32(st, d, L, Qall, L, QTall));
    Qb = Qall;
    QT32 = QTall;
  }
  const int64_t Lp = cdiv(L, 16) * 16;
  // Rayleigh-Ritz: Wq = X Q (n x L), B = Wq^T Wq / n (FP64), B = V diag(theta) V^T
  WS(Wq, float, std::string("Wq") + ksfx, (size_t)n * Lp);
  SCS_CHECK(launch_gemm_nt_longk(st, bf, X, n, d, ldx, QT32, L, d, Wq, Lp, true));
  // in FP32 with L <= 64 the narrow Gram kernel (slabs of X Q staged in LDS); else the split-K TN GEMM
  const bool narrow = !bf && L <= 64;
  int64_t nch2 = narrow ? gram_rr_f32_parts(n) : gemm_tn_splitk_chunks(n, L, L, Wq, Lp, Wq, Lp);
  int64_t chunk2 = cdiv(n, nch2);
  if (!narrow) nch2 = cdiv(n, chunk2);
  WS(part2, float, std::string("partial2") + sfx, (size_t)nch2 * L * L);
  if (narrow) SCS_CHECK(launch_gram_rr_f32(st, Wq, n, L, Lp, part2));
  else SCS_CHECK(launch_gemm_tn_splitk(st, bf, Wq, n, L, Lp, Wq, L, Lp, part2, chunk2, nch2));
  WS(B, double, std::string("B64") + ksfx, (size_t)L * L);
  SCS_CHECK(launch_reduce_partials_f64(st, part2, nch2, (int64_t)L * L, 1.0 / (double)n, B));
  // the sketch reads X no more, and what follows is mostly one-workgroup FP64 algebra: work forked
  // here overlaps it (forked before this reduce, a gradient pass slowed the reduce down fourfold)
  if (x_done) SCS_HIP(hipEventRecord(x_done, st));
  if (split) {
    split->B = B;
    split->Q = Qb;
    split->L = L;
    split->Wq = Wq;
    split->Lp = Lp;
    return SCS_OK;
  }
  WS(V, double, std::string("V64") + sfx, (size_t)L * L);
  WS(theta, double, std::string("theta") + sfx, (size_t)L);
  WS(order, int, std::string("order") + sfx, (size_t)L);
  WS(eigw, double, std::string("eig_work") + sfx, eig64_work_len(L));
  SCS_CHECK(launch_eig64(st, B, L, eigw, V, theta, order));
  // lift: U~ = Q V_k, lam = theta_{1..k}
  WS(U64, double, std::string("U64") + sfx, (size_t)d * k);
  WS(U32, float, std::string("U32") + sfx, (size_t)d * k);
  WS(UT32, float, std::string("UT32") + sfx, (size_t)k * d);
  WS(lam, double, std::string("lam") + sfx, (size_t)k);
  WS(VkT, float, std::string("VkT") + sfx, (size_t)k * L);
  SCS_CHECK(launch_lift(st, Qb, d, L, V, order, k, theta, U64, U32, UT32, lam, VkT));
  if (want_z) {
    const int64_t kz = gemm_wide_kpad(k);
    WS(Z, float, std::string("Z") + sfx, (size_t)n * kz);
    SCS_CHECK(launch_gemm_nt_longk(st, bf, Wq, n, L, Lp, VkT, k, L, Z, kz, true));
  }
  if (flags_out) return SCS_OK;
  int hflags[2] = {0, 0};
  SCS_HIP(hipMemcpyAsync(hflags, flags, sizeof(hflags), hipMemcpyDeviceToHost, st));
  SCS_HIP(hipStreamSynchronize(st));
  *rank_def = hflags[0] || hflags[1];
  return SCS_OK;
}

// Preconditioned rows: Xt = X/s + Z (U D)^T (ld ldt), reg = sqrt(n lambda)(U (U D)^T + I/s), beta = row norms.
// Z: n x k with leading dimension gemm_wide_kpad(k), zero up to the next multiple of 16.
// Events for work forked onto side stream 0 inside one call (fork slot i: fork_ev[i] / join_ev[i]).
int ensure_fork_events(scs_ctx* c) {
  for (int i = 0; i < 2; ++i) {
    if (!c->fork_ev[i]) SCS_HIP(hipEventCreateWithFlags(&c->fork_ev[i], hipEventDisableTiming));
    if (!c->join_ev[i]) SCS_HIP(hipEventCreateWithFlags(&c->join_ev[i], hipEventDisableTiming));
  }
  return ensure_side_streams(c, 1);
}

// Preconditioned rows: Xt = X/s + Z (U D)^T (ld ldt), reg = sqrt(n lambda)(U (U D)^T + I/s), beta = row norms.
// Z: n x k with leading dimension gemm_wide_kpad(k), zero up to the next multiple of 16.
// aux (nullable): a second stream for the regularizer rows, which then run beside the data rows (the
// caller's stream waits for them before returning from this enqueue sequence's join).
int apply_impl(scs_ctx* ctx, const float* X, int64_t n, int64_t d, int64_t ldx, const float* U32, const float* Z,
               const double* lam, int k, double lambda, int gemm_bf16, int out_bf16, void* Xt, void* reg,
               int64_t ldt, float* beta, SolveState* state, hipStream_t st_in = nullptr, const std::string& sfx = "",
               bool fork_reg = false) {
  hipStream_t st = st_in ? st_in : ctx->stream;
  const int64_t kz = gemm_wide_kpad(k), drows = gemm_wide_bt_rows(d);
  WS(UD, float, "UD32" + sfx, (size_t)drows * kz);
  WS(Up, float, "Upad32" + sfx, (size_t)drows * kz);
  WS(scal, double, "scal" + sfx, 2);
  SCS_CHECK(launch_precond_setup(st, lam, k, lambda, n, U32, d, UD, Up, kz, scal, state));
  hipStream_t rs = st;
  if (fork_reg) {  // the d x d regularizer GEMM fills few CUs: run it beside the n x d one
    SCS_CHECK(ensure_fork_events(ctx));
    rs = ctx->side[0];
    SCS_HIP(hipEventRecord(ctx->fork_ev[1], st));
    SCS_HIP(hipStreamWaitEvent(rs, ctx->fork_ev[1], 0));
  }
  SCS_CHECK(launch_gemm_nt_wide(rs, gemm_bf16, Up, d, k, kz, UD, d, kz, (float)std::sqrt((double)n * lambda),
                                nullptr, 0, 0.f, nullptr, 0.f, scal + 1, out_bf16, reg, ldt, beta ? beta + n : nullptr));
  SCS_CHECK(launch_gemm_nt_wide(st, gemm_bf16, Z, n, k, kz, UD, d, kz, 1.0f, X, ldx, 0.f, scal, 0.f, nullptr,
                                out_bf16, Xt, ldt, beta));
  if (fork_reg) {
    SCS_HIP(hipEventRecord(ctx->join_ev[1], rs));
    SCS_HIP(hipStreamWaitEvent(st, ctx->join_ev[1], 0));
  }
  return SCS_OK;
}

int validate_problem(const void* X, int64_t n, int64_t d, int64_t ldx, double lambda) {
  if (!X) {
    set_error("null X");
    return SCS_EINVAL;
  }
  if (n < 1 || d < 1 || ldx < d) {
    set_error("need n >= 1, d >= 1, ldx >= d");
    return SCS_EINVAL;
  }
  if (!(lambda > 0.0) || !std::isfinite(lambda)) {
    set_error("lambda must be a finite positive number");
    return SCS_EINVAL;
  }
  return SCS_OK;
}

}  // namespace

extern "C" {

void scs_opts_default(scs_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->oversample = 5;
  o->batch = 64;
  o->steps = 0;
  o->step_scale = 1.0;
  o->max_epochs = 30;
  o->stop_rule = SCS_STOP_CERTIFICATE;
  o->f_star = 0.0;
  o->average = 1;
  o->precision = SCS_PREC_FP32;
  o->workgroups = 0;
  o->seed = 20160207ull;
}

const char* scs_status_string(int s) {
  switch (s) {
    case SCS_OK: return "ok";
    case SCS_EINVAL: return "invalid argument";
    case SCS_ENONFINITE: return "non-finite value in X or y";
    case SCS_ENOMEM: return "device allocation failed";
    case SCS_EDEVICE: return "HIP runtime error";
    case SCS_NOT_CONVERGED: return "epoch cap reached before the stop rule held";
    case SCS_DIVERGED: return "diverged; returned the last good snapshot";
    case SCS_SKETCH_RANK_DEFICIENT: return "sketch lost rank; solved without preconditioning";
  }
  return "unknown status";
}

const char* scs_last_error(void) { return g_last_error.c_str(); }

int scs_create(scs_ctx** out, int device, void* hip_stream) {
  if (!out) return SCS_EINVAL;
  *out = nullptr;
  int ndev = 0;
  SCS_HIP(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) {
    set_error("no such HIP device");
    return SCS_EINVAL;
  }
  {
    Guard g(device);
    // device address of the allocation-free entry point's fixed scratch array on this device
    SCS_CHECK(noalloc_scratch_init(device));
  }
  auto* c = new scs_ctx();
  c->device = device;
  if (const char* e = std::getenv("SCS_XCD_STRIDE")) c->xcd_stride = std::max(1, std::atoi(e));
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  *out = c;
  return SCS_OK;
}

int scs_destroy(scs_ctx* c) {
  if (!c) return SCS_OK;
  Guard g(c->device);
  hipStreamSynchronize(c->stream);
  for (auto q : c->side) hipStreamSynchronize(q);
  free_retired(c);
  for (auto& kv : c->bufs)
    if (kv.second.p) hipFree(kv.second.p);
  for (auto e : c->events) hipEventDestroy(e);
  for (auto e : c->tevents) hipEventDestroy(e);
  for (auto e : c->side_events) hipEventDestroy(e);
  for (auto q : c->side) hipStreamDestroy(q);
  for (auto e : c->tune_ev)
    if (e) hipEventDestroy(e);
  if (c->stop_flags) hipHostFree(c->stop_flags);
  delete c;
  return SCS_OK;
}

int scs_gaussian(scs_ctx* ctx, uint64_t seed, int64_t count, float* out) {
  if (!ctx || !out || count < 0) return SCS_EINVAL;
  Guard g(ctx->device);
  free_retired(ctx);
  return launch_gaussian(ctx->stream, seed, count, out);
}

int scs_sample_indices(scs_ctx* ctx, const float* beta, int64_t N, uint64_t seed, int epoch, int64_t count,
                       int32_t* out) {
  if (!ctx || !beta || !out || N < 1 || count < 0 || N > INT32_MAX) return SCS_EINVAL;
  Guard g(ctx->device);
  free_retired(ctx);
  WS(cum, uint64_t, "cum", (size_t)N);
  WS(scr, double, "sampler_scratch", (size_t)sampler_scratch_len(N));
  SCS_CHECK(launch_sampler_prepare(ctx->stream, beta, N, cum, scr, sampler_scratch_len(N), nullptr));
  return launch_sample(ctx->stream, cum, N, N, seed, epoch, count, count, out, static_cast<float*>(nullptr), nullptr);
}

int scs_sketch_build(scs_ctx* ctx, const float* X, int64_t n, int64_t d, int64_t ldx, int k, const scs_opts* opts,
                     float* U_out, double* U64_out, double* lam_out) {
  if (!ctx || !U_out || !lam_out) return SCS_EINVAL;
  SCS_CHECK(validate_problem(X, n, d, ldx, 1.0));
  scs_opts o;
  scs_opts_default(&o);
  if (opts) o = *opts;
  const int l = k + o.oversample;
  if (k < 1 || k > d || o.oversample < 0 || !sketch_width_ok(o, k, n, d)) {
    set_error("sketch: need 1 <= k, q (k + p) <= min(d, n, 136) for q Krylov blocks");
    return SCS_EINVAL;
  }
  Guard g(ctx->device);
  free_retired(ctx);
  bool rd = false;
  SCS_CHECK(sketch_impl(ctx, X, n, d, ldx, k, o, false, &rd));
  hipStream_t st = ctx->stream;
  SCS_HIP(hipMemcpyAsync(U_out, ws<float>(ctx, "U32", 0), sizeof(float) * d * k, hipMemcpyDeviceToDevice, st));
  if (U64_out)
    SCS_HIP(hipMemcpyAsync(U64_out, ws<double>(ctx, "U64", 0), sizeof(double) * d * k, hipMemcpyDeviceToDevice, st));
  SCS_HIP(hipMemcpyAsync(lam_out, ws<double>(ctx, "lam", 0), sizeof(double) * k, hipMemcpyDeviceToDevice, st));
  SCS_HIP(hipStreamSynchronize(st));
  return rd ? SCS_SKETCH_RANK_DEFICIENT : SCS_OK;
}

int scs_precondition_apply(scs_ctx* ctx, const float* X, int64_t n, int64_t d, int64_t ldx, const float* U,
                           const double* lam, int k, double lambda, int xt_bf16, void* Xt_out, void* reg_out,
                           int64_t ldt, float* beta_out) {
  if (!ctx || !Xt_out || !reg_out || ldt < d || k < 0 || k > d || (k > 0 && (!U || !lam))) return SCS_EINVAL;
  SCS_CHECK(validate_problem(X, n, d, ldx, lambda));
  if (k > 160) {
    set_error("apply: k > 160");
    return SCS_EINVAL;
  }
  Guard g(ctx->device);
  free_retired(ctx);
  hipStream_t st = ctx->stream;
  if (k == 0) {
    // P = I: x~_i = x_i, rows sqrt(n lambda) e_j
    WS(I1, double, "unit_lam", 1);
    (void)I1;
    if (xt_bf16) {
      WS(tmp, uint16_t, "xcopy16", (size_t)n * d);
      SCS_CHECK(launch_copy_bf16(st, X, n, d, ldx, tmp));
      SCS_HIP(hipMemcpy2DAsync(Xt_out, ldt * 2, tmp, d * 2, d * 2, n, hipMemcpyDeviceToDevice, st));
      if (beta_out) SCS_CHECK(launch_rownorm_bf16(st, tmp, n, d, beta_out));
    } else {
      SCS_HIP(hipMemcpy2DAsync(Xt_out, ldt * 4, X, ldx * 4, d * 4, n, hipMemcpyDeviceToDevice, st));
      if (beta_out) SCS_CHECK(launch_rownorm(st, X, n, d, ldx, beta_out));
    }
    WS(tmpreg, float, "regtmp", (size_t)d * d);
    SCS_CHECK(launch_fill_scaled_identity(st, d, std::sqrt((double)n * lambda), xt_bf16, tmpreg,
                                          beta_out ? beta_out + n : nullptr));
    SCS_HIP(hipMemcpy2DAsync(reg_out, ldt * (xt_bf16 ? 2 : 4), tmpreg, d * (xt_bf16 ? 2 : 4), d * (xt_bf16 ? 2 : 4), d,
                             hipMemcpyDeviceToDevice, st));
    return SCS_OK;
  }
  WS(UT, float, "UT_apply", (size_t)k * d);
  SCS_CHECK(launch_transpose_f32(st, U, d, k, UT));
  const int64_t kz = gemm_wide_kpad(k);
  WS(Z, float, "Z_apply", (size_t)n * kz);
  SCS_CHECK(launch_gemm_nt_longk(st, xt_bf16, X, n, d, ldx, UT, k, d, Z, kz, true));
  return apply_impl(ctx, X, n, d, ldx, U, Z, lam, k, lambda, xt_bf16, xt_bf16, Xt_out, reg_out, ldt, beta_out,
                    nullptr);
}

int scs_full_gradient(scs_ctx* ctx, const float* X, int64_t n, int64_t d, int64_t ldx, const float* y,
                      const float* U, const double* lam, int k, double lambda, const float* wt, float* grad_out,
                      double* obj_out) {
  if (!ctx || !y || !wt || !grad_out || k < 0 || k > d || (k > 0 && (!U || !lam))) return SCS_EINVAL;
  SCS_CHECK(validate_problem(X, n, d, ldx, lambda));
  if (k > 256) return SCS_EINVAL;
  Guard g(ctx->device);
  free_retired(ctx);
  hipStream_t st = ctx->stream;
  const float* UT = nullptr;
  if (k > 0) {
    WS(ut, float, "UT_grad", (size_t)k * d);
    SCS_CHECK(launch_transpose_f32(st, U, d, k, ut));
    UT = ut;
  }
  WS(state, SolveState, "state_grad", 1);
  SCS_HIP(hipMemsetAsync(state, 0, sizeof(SolveState), st));
  WS(w32, float, "w32_grad", (size_t)d);
  WS(tmp, double, "vtmp", (size_t)d);
  WS(g64, double, "g64", (size_t)16 * d);  // kColSplit x d first-level gradient sums
  int nwg = grad_num_workgroups(n, d);
  WS(part, float, "gpart", (size_t)nwg * d);
  WS(rsq, double, "grsq", (size_t)nwg);
  SCS_CHECK(launch_premap(st, UT, U, lam, k, d, lambda, wt, w32, nullptr, tmp, state));
  SCS_CHECK(launch_grad_partial(st, X, n, d, ldx, y, w32, part, rsq, nwg, state));
  WS(wcur, float, "wt_dummy", (size_t)d);
  SCS_CHECK(launch_grad_finish(st, part, rsq, nwg, n, d, w32, lambda, UT, U, lam, k, grad_out, g64, tmp, state,
                               SCS_STOP_EPOCHS, 0.0, 0.0, wcur, nullptr, 1, nullptr));
  SolveState hs;
  SCS_HIP(hipMemcpyAsync(&hs, state, sizeof(hs), hipMemcpyDeviceToHost, st));
  SCS_HIP(hipStreamSynchronize(st));
  if (obj_out) *obj_out = hs.obj0;
  if (hs.status == SCS_ENONFINITE) return SCS_ENONFINITE;
  return SCS_OK;
}

int scs_regularization_for_budget(scs_ctx* ctx, const float* X, int64_t n, int64_t d, int64_t ldx, int k,
                                  const scs_opts* opts, double* lambda_precond, double* lambda_plain) {
  if (!ctx || !lambda_precond || !lambda_plain) return SCS_EINVAL;
  SCS_CHECK(validate_problem(X, n, d, ldx, 1.0));
  scs_opts o;
  scs_opts_default(&o);
  if (opts) o = *opts;
  const int l = k + o.oversample;
  if (k < 1 || k > d || o.oversample < 0 || !sketch_width_ok(o, k, n, d)) {
    set_error("budget regularization: need 1 <= k, q (k + p) <= min(d, n, 136) for q Krylov blocks");
    return SCS_EINVAL;
  }
  Guard g(ctx->device);
  free_retired(ctx);
  hipStream_t st = ctx->stream;
  bool rd = false;
  SCS_CHECK(sketch_impl(ctx, X, n, d, ldx, k, o, false, &rd));
  // ||X||_F^2 in FP64: the sampler's sum of the FP32 row norms
  WS(rn, float, "budget_rownorm", (size_t)n);
  WS(cum, uint64_t, "budget_cum", (size_t)n);
  WS(scr, double, "sampler_scratch", (size_t)sampler_scratch_len(n));
  WS(state, SolveState, "budget_state", 1);
  WS(out, double, "budget_out", 2);
  SCS_CHECK(launch_zero3(st, state, (int64_t)sizeof(SolveState), nullptr, 0, nullptr, 0));
  SCS_CHECK(launch_rownorm(st, X, n, d, ldx, rn));
  SCS_CHECK(launch_sampler_prepare(st, rn, n, cum, scr, sampler_scratch_len(n), state));
  SCS_CHECK(launch_budget_lambda(st, ws<double>(ctx, "lam", 0), k, state, n, out));
  double h[2] = {0.0, 0.0};
  SCS_HIP(hipMemcpyAsync(h, out, sizeof(h), hipMemcpyDeviceToHost, st));
  SCS_HIP(hipStreamSynchronize(st));
  *lambda_precond = h[0];
  *lambda_plain = h[1];
  return rd ? SCS_SKETCH_RANK_DEFICIENT : SCS_OK;
}

int scs_full_gradient_noalloc(scs_ctx* ctx, const float* X, int64_t n, int64_t d, int64_t ldx, const float* y,
                              const float* U, const double* lam, int k, double lambda, const float* wt,
                              float* grad_out, double* obj_out) {
  if (!ctx || !y || !wt || !grad_out || k < 0 || k > d || (k > 0 && (!U || !lam))) return SCS_EINVAL;
  SCS_CHECK(validate_problem(X, n, d, ldx, lambda));
  if (k > 256) return SCS_EINVAL;
  Guard g(ctx->device);
  return full_gradient_noalloc(ctx->device, ctx->stream, X, n, d, ldx, y, U, lam, k, lambda, wt, grad_out, obj_out);
}

int scs_svrg_epoch(scs_ctx* ctx, int64_t n, int64_t d, const void* Xt, const void* reg, int64_t ldt, int xt_bf16,
                   const float* beta, const float* mu, const int32_t* idx, int64_t m, int b, double eta, int average,
                   int workgroups, int wave_rows, float* wt) {
  if (!ctx || !Xt || !reg || !beta || !mu || !idx || !wt || n < 1 || d < 1 || ldt < d || ldt % 4 != 0 || m < 1 ||
      b < 1 || b > kInnerMaxB || !(eta > 0.0))
    return SCS_EINVAL;
  Guard g(ctx->device);
  free_retired(ctx);
  hipStream_t st = ctx->stream;
  const int64_t N = n + d;
  WS(cum, uint64_t, "cum", (size_t)N);
  WS(scr, double, "sampler_scratch", (size_t)sampler_scratch_len(N));
  WS(state, SolveState, "state_epoch", 1);
  SCS_HIP(hipMemsetAsync(state, 0, sizeof(SolveState), st));
  SCS_CHECK(launch_sampler_prepare(st, beta, N, cum, scr, sampler_scratch_len(N), state));
  WS(scale, float, "scale", (size_t)m * b);
  SCS_CHECK(launch_index_scale(st, cum, N, n, idx, m * b, scale, state));
  scs_opts o;
  scs_opts_default(&o);
  o.workgroups = workgroups;
  o.batch = b;
  const int W = choose_workgroups(o, d);
  WS(xbuf, uint64_t, "xbuf", (size_t)inner_xbuf_words(W));
  SCS_HIP(hipMemsetAsync(xbuf, 0, sizeof(uint64_t) * inner_xbuf_words(W), st));
  InnerArgs a{};
  a.n = n;
  a.d = d;
  a.Xt = Xt;
  a.ldx = ldt;
  a.reg = reg;
  a.ldr = ldt;
  a.mu = mu;
  a.idx = idx;
  a.scale = scale;
  a.m = m;
  a.b = b;
  a.eta = eta;
  a.eta_from_state = 0;
  a.average = average;
  a.W = W;
  a.xcd_stride = W > 1 ? ctx->xcd_stride : 1;
  a.step_base = 0;
  a.wt = wt;
  a.wt_prev = nullptr;
  a.xbuf = xbuf;
  a.state = state;
  a.wave_rows = wave_rows;
  SCS_CHECK(launch_inner_epoch(st, a, xt_bf16));
  SolveState hs;
  SCS_HIP(hipMemcpyAsync(&hs, state, sizeof(hs), hipMemcpyDeviceToHost, st));
  SCS_HIP(hipStreamSynchronize(st));
  if (hs.status == SCS_EDEVICE) {
    set_error("inner loop: a cross-workgroup wait exceeded its budget");
    return SCS_EDEVICE;
  }
  return SCS_OK;
}

// The single solve. CholeskyQR's breakdown flags are written to host-pinned memory and read at the
// first stop decision, so the host never waits for the sketch: in the rare breakdown case the work
// queued so far is discarded and the solve runs again with P = I (sketch_failed), reporting
// SCS_SKETCH_RANK_DEFICIENT as before.
static int svrg_solve_impl(scs_ctx* ctx, const float* X, int64_t n, int64_t d, int64_t ldx, const float* y,
                           double lambda, int k, double eps, const scs_opts* opts, float* w_out, scs_report* report,
                           bool sketch_failed) {
  if (!ctx || !y || !w_out) {
    set_error("null argument");
    return SCS_EINVAL;
  }
  SCS_CHECK(validate_problem(X, n, d, ldx, lambda));
  scs_opts o;
  scs_opts_default(&o);
  if (opts) o = *opts;
  const int l = k + o.oversample;
  if (k < 0 || k > d || (k > 0 && (o.oversample < 0 || !sketch_width_ok(o, k, n, d)))) {
    set_error("need 0 <= k and, for k > 0, q (k + p) <= min(d, n, 136) for q Krylov blocks");
    return SCS_EINVAL;
  }
  if (o.batch < 1 || o.batch > kInnerMaxB || o.max_epochs < 1 || o.steps < 0 || !(o.step_scale > 0.0) ||
      !(o.epoch_factor >= 0.0) || o.stop_rule < 0 || o.stop_rule > 2 || n + d > INT32_MAX || o.epoch_offset < 0 ||
      (k > 256 && o.w0 && !o.w0_preconditioned)) {
    set_error("bad options: need 1 <= batch <= 256, max_epochs >= 1, steps >= 0, step_scale > 0, epoch_offset >= 0");
    return SCS_EINVAL;
  }
  Guard g(ctx->device);
  free_retired(ctx);
  hipStream_t st = ctx->stream;
  const int b = o.batch;
  const int64_t m = epoch_steps(o, n, b);
  const int64_t N = n + d;
  const int S = o.max_epochs;
  const int mixed = o.precision == SCS_PREC_MIXED;
  // rows used by the inner loop start on 256-byte boundaries, so a workgroup's column slice of a
  // gathered row covers whole cache lines
  const int64_t ldt = cdiv(d, mixed ? 128 : 64) * (mixed ? 128 : 64);
  // Events (each one recorded between two kernels costs a few microseconds of dispatch, so an epoch
  // records one, or more only when timing is asked for): 0 start, 1 sketch done, 2 preconditioner
  // done, 3 end of solve, 4 + s end of epoch s (also the point where the host reads the stop flag of
  // snapshot s); with timing >= 1, 6 + 3S + s opens the inner loop of s; with timing >= 2,
  // 4 + S + s and 5 + 2S + s bracket the gradient pass of s.
  SCS_CHECK(ensure_events(ctx, 0, (size_t)(o.timing ? 6 + 4 * S : 4 + S)));
  // host-pinned: S + 1 stop flags, then CholeskyQR's two breakdown flags
  SCS_CHECK(ensure_stop_flags(ctx, (size_t)S + 3));
  std::memset(ctx->stop_flags, 0, sizeof(int) * (S + 3));
  int* chol_flags = ctx->stop_flags + S + 1;
  hipEvent_t* tev = ctx->tevents.data();
  hipEvent_t ev_start = tev[0], ev_sketch = tev[1], ev_apply = tev[2], ev_end = tev[3];
  auto ev_epoch = [&](int s) { return tev[4 + s]; };
  auto ev_g0 = [&](int s) { return tev[4 + S + s]; };
  auto ev_g1 = [&](int s) { return tev[5 + 2 * S + s]; };
  auto ev_i0 = [&](int s) { return tev[6 + 3 * S + s]; };
  SCS_HIP(hipEventRecord(ev_start, st));

  WS(state, SolveState, "state", 1);
  SCS_HIP(hipMemsetAsync(state, 0, sizeof(SolveState), st));
  WS(w32, float, "w32", (size_t)d);
  const int nwg = grad_num_workgroups(n, d);
  WS(gpart, float, "gpart", (size_t)nwg * d);
  WS(grsq, double, "grsq", (size_t)nwg);

  // The first snapshot is w~ = 0 (no start point given), so w = P^{-1/2} w~ = 0 and the first gradient
  // pass does not depend on the sketch: it runs on a side stream while the sketch's one-workgroup FP64
  // kernels occupy one CU (after the sketch's last pass over X), and is joined before the first gradient
  // finish. (Not with timing >= 2, which brackets every pass with events on the solve's stream.)
  const bool early_grad = !sketch_failed && k > 0 && !o.w0 && o.timing < 2;
  if (early_grad) SCS_CHECK(ensure_fork_events(ctx));

  // ---- sketch (Alg. 3, Block Lanczos step)
  int k_used = sketch_failed ? 0 : k;
  const bool rank_def = sketch_failed;
  if (k_used > 0)
    SCS_CHECK(sketch_impl(ctx, X, n, d, ldx, k, o, true, nullptr, chol_flags, nullptr, "",
                          early_grad ? ctx->fork_ev[0] : nullptr));
  if (early_grad) {
    // forked once the sketch has finished streaming X, so that it overlaps the sketch's FP64 algebra
    hipStream_t gs = ctx->side[0];
    SCS_HIP(hipStreamWaitEvent(gs, ctx->fork_ev[0], 0));
    SCS_CHECK(launch_zero3(gs, w32, (int64_t)sizeof(float) * d, nullptr, 0, nullptr, 0));
    SCS_CHECK(launch_grad_partial(gs, X, n, d, ldx, y, w32, gpart, grsq, nwg, state));
    SCS_HIP(hipEventRecord(ctx->join_ev[0], gs));
  }
  auto sketch_broke = [&]() {
    return k_used > 0 && (__atomic_load_n(chol_flags, __ATOMIC_ACQUIRE) || __atomic_load_n(chol_flags + 1, __ATOMIC_ACQUIRE));
  };
  SCS_HIP(hipEventRecord(ev_sketch, st));

  // ---- preconditioned rows and smoothness (Alg. 3, x~_i, b_j, beta_i)
  WS(beta, float, "beta", (size_t)N);
  const void* Xt = nullptr;
  int64_t ldxt = ldt;
  int rows_bf16 = mixed;
  const float* U32 = nullptr;
  const float* UT32 = nullptr;
  const double* lam = nullptr;
  if (k_used > 0) {
    void* xt = wsb(ctx, "Xt", (size_t)n * ldt * (mixed ? 2 : 4));
    void* rg = wsb(ctx, "reg", (size_t)d * ldt * (mixed ? 2 : 4));
    if (!xt || !rg) return SCS_ENOMEM;
    U32 = ws<float>(ctx, "U32", 0);
    UT32 = ws<float>(ctx, "UT32", 0);
    lam = ws<double>(ctx, "lam", 0);
    SCS_CHECK(apply_impl(ctx, X, n, d, ldx, U32, ws<float>(ctx, "Z", 0), lam, k_used, lambda, mixed, mixed, xt, rg,
                         ldt, beta, state, nullptr, "", true));
    Xt = xt;
  } else {
    if (mixed) {
      WS(xt16, uint16_t, "Xt16", (size_t)n * ldt);
      WS(tmp, uint16_t, "xcopy16", (size_t)n * d);
      SCS_CHECK(launch_copy_bf16(st, X, n, d, ldx, tmp));
      SCS_HIP(hipMemcpy2DAsync(xt16, ldt * 2, tmp, d * 2, d * 2, n, hipMemcpyDeviceToDevice, st));
      SCS_CHECK(launch_rownorm_bf16(st, tmp, n, d, beta));
      Xt = xt16;
    } else {
      // P = I: the rows are x_i themselves, copied into the padded layout of the inner loop
      WS(xpad, float, "Xpad", (size_t)n * ldt);
      SCS_HIP(hipMemcpy2DAsync(xpad, ldt * 4, X, ldx * 4, d * 4, n, hipMemcpyDeviceToDevice, st));
      SCS_CHECK(launch_rownorm(st, X, n, d, ldx, beta));
      Xt = xpad;
    }
  }
  // regularizer rows share the data rows' leading dimension (the inner loop addresses both from one stride)
  void* reg = nullptr;
  if (k_used > 0) {
    reg = ws<char>(ctx, "reg", 0);
  } else {
    WS(rtmp, float, "regtmp", (size_t)d * d);
    SCS_CHECK(launch_fill_scaled_identity(st, d, std::sqrt((double)n * lambda), mixed, rtmp, beta + n));
    reg = wsb(ctx, "reg", (size_t)d * ldxt * (mixed ? 2 : 4));
    if (!reg) return SCS_ENOMEM;
    SCS_HIP(hipMemcpy2DAsync(reg, ldxt * (mixed ? 2 : 4), rtmp, d * (mixed ? 2 : 4), d * (mixed ? 2 : 4), d,
                             hipMemcpyDeviceToDevice, st));
  }
  // ---- sampling weights (Alg. 1: q_i = beta_i / sum beta)
  WS(cum, uint64_t, "cum", (size_t)N);
  WS(scr, double, "sampler_scratch", (size_t)sampler_scratch_len(N));
  SCS_CHECK(launch_sampler_prepare(st, beta, N, cum, scr, sampler_scratch_len(N), state, o.uniform_sampling));
  SCS_HIP(hipEventRecord(ev_apply, st));

  // ---- SVRG epochs (Alg. 1)
  int W = choose_workgroups(o, d);
  WS(wt, float, "wt", (size_t)d);
  WS(wt_prev, float, "wt_prev", (size_t)d);
  WS(mu, float, "mu", (size_t)d);
  WS(tmp, double, "vtmp", (size_t)d);
  WS(g64, double, "g64", (size_t)16 * d);  // kColSplit x d first-level gradient sums
  // index streams are drawn kSampleGroup epochs per launch
  constexpr int kSampleGroup = 8;
  WS(idxb, int32_t, "idx", (size_t)kSampleGroup * m * b);
  WS(scale, float, "scale", (size_t)kSampleGroup * m * b);
  WS(xbuf, uint64_t, "xbuf", (size_t)inner_xbuf_words(16));
  SCS_CHECK(launch_zero3(st, wt, (int64_t)sizeof(float) * d, wt_prev, (int64_t)sizeof(float) * d, xbuf,
                         (int64_t)sizeof(uint64_t) * inner_xbuf_words(16)));
  if (o.w0) {
    // start point: the solver's variable as given, or w~ = P^{1/2} w0 (P = I when k = 0)
    if (o.w0_preconditioned || k_used == 0)
      SCS_HIP(hipMemcpyAsync(wt, o.w0, sizeof(float) * d, hipMemcpyDeviceToDevice, st));
    else
      SCS_CHECK(launch_pmhalf_inv(st, UT32, lam, k_used, d, lambda, o.w0, wt));
    SCS_HIP(hipMemcpyAsync(wt_prev, wt, sizeof(float) * d, hipMemcpyDeviceToDevice, st));
  }

  InnerArgs a{};
  a.n = n;
  a.d = d;
  a.Xt = Xt;
  a.ldx = ldxt;
  a.reg = reg;
  a.ldr = ldxt;
  a.mu = mu;
  a.scale = scale;
  a.m = m;
  a.b = b;
  a.eta_from_state = 1;
  a.step_scale = o.step_scale;
  a.average = o.average;
  a.W = W;
  a.xcd_stride = W > 1 ? ctx->xcd_stride : 1;
  a.wt = wt;
  a.wt_prev = wt_prev;
  a.xbuf = xbuf;
  a.state = state;
  a.wave_rows = o.wave_rows;
  if (o.wave_rows == kInnerLookahead && o.workgroups <= 0) {
    // the look-ahead loop takes slices of at most 64 columns
    W = (int)std::max<int64_t>(1, cdiv(d, 64));
    a.W = W;
    a.xcd_stride = W > 1 ? ctx->xcd_stride : 1;
  } else if (o.workgroups < 0) {
    int wr = 0;
    SCS_CHECK(autotune_workgroups(ctx, st, a, rows_bf16, cum, N, o.seed, &W, &wr));
    a.W = W;
    a.xcd_stride = W > 1 ? ctx->xcd_stride : 1;
    if (o.wave_rows == 0) a.wave_rows = wr;
  }

  constexpr int kLookahead = 3;
  int last_epoch = -1;
  bool redo = false;
  // an event per epoch only where its time is asked for: recording one costs a few microseconds of
  // dispatch between two epochs, and the host's stop check waits on the flag itself
  const bool epoch_events = o.epoch_ms != nullptr || o.timing != 0;
  for (int s = 0; s <= S; ++s) {
    float* trace_row = (o.trace_w && s < S) ? o.trace_w + (int64_t)s * d : nullptr;
    if (s == 0 && early_grad) {
      // the pass at w = 0 already ran beside the sketch
      if (trace_row) SCS_CHECK(launch_zero3(st, trace_row, (int64_t)sizeof(float) * d, nullptr, 0, nullptr, 0));
      SCS_HIP(hipStreamWaitEvent(st, ctx->join_ev[0], 0));
    } else {
      SCS_CHECK(launch_premap(st, UT32, U32, lam, k_used, d, lambda, wt, w32, trace_row, tmp, state));
      if (o.timing >= 2) SCS_HIP(hipEventRecord(ev_g0(s), st));
      SCS_CHECK(launch_grad_partial(st, X, n, d, ldx, y, w32, gpart, grsq, nwg, state));
      if (o.timing >= 2) SCS_HIP(hipEventRecord(ev_g1(s), st));
    }
    SCS_CHECK(launch_grad_finish(st, gpart, grsq, nwg, n, d, w32, lambda, UT32, U32, lam, k_used, mu, g64, tmp, state,
                                 o.stop_rule, eps, o.f_star, wt, wt_prev, s == 0 ? 1 : 0, ctx->stop_flags + s));
    if (s == S) break;
    const int64_t mb = m * b, slot = s % kSampleGroup;
    if (slot == 0) {
      const int64_t cnt = (int64_t)std::min(kSampleGroup, S - s) * mb;
      if (o.indices) SCS_CHECK(launch_index_scale(st, cum, N, n, o.indices + (int64_t)s * mb, cnt, scale, state));
      else SCS_CHECK(launch_sample(st, cum, N, n, o.seed, s + o.epoch_offset, mb, cnt, idxb, scale, state));
    }
    a.idx = o.indices ? o.indices + (int64_t)s * mb : idxb + slot * mb;
    a.scale = scale + slot * mb;
    a.step_base = (uint32_t)((uint64_t)s * (uint64_t)m);
    if (o.timing) SCS_HIP(hipEventRecord(ev_i0(s), st));
    SCS_CHECK(launch_inner_epoch(st, a, rows_bf16));
    if (epoch_events) SCS_HIP(hipEventRecord(ev_epoch(s), st));
    last_epoch = s;
    // Keep kLookahead epochs queued ahead of the host's view: once the stop flag of snapshot
    // s - kLookahead + 1 (written before that epoch's inner loop) says the solve is finished, the
    // epochs already queued after it are no-ops (every kernel returns on the device's done flag) and
    // nothing more is enqueued.
    if (s + 1 >= kLookahead) {
      const int q = s + 1 - kLookahead;
      int flag = 0;
      SCS_CHECK(wait_stop_flag(ctx, st, q, &flag));
      if (sketch_broke()) {
        redo = true;
        break;
      }
      if (flag == 1) break;
    }
  }
  // w = P^{-1/2} w~ with the same routine that produced the gradient's evaluation point
  SCS_CHECK(launch_premap(st, UT32, U32, lam, k_used, d, lambda, wt, w_out, nullptr, tmp, nullptr));
  if (o.wt_out) SCS_HIP(hipMemcpyAsync(o.wt_out, wt, sizeof(float) * d, hipMemcpyDeviceToDevice, st));
  SCS_HIP(hipEventRecord(ev_end, st));
  SolveState hs;
  SCS_HIP(hipMemcpyAsync(&hs, state, sizeof(hs), hipMemcpyDeviceToHost, st));
  SCS_HIP(hipStreamSynchronize(st));
  if (redo || sketch_broke())
    return svrg_solve_impl(ctx, X, n, d, ldx, y, lambda, k, eps, opts, w_out, report, true);

  int status = SCS_OK;
  if (hs.status == SCS_ENONFINITE || hs.status == SCS_EDEVICE) {
    if (hs.status == SCS_EDEVICE) set_error("inner loop: a cross-workgroup wait exceeded its budget");
    else set_error("non-finite value in X or y");
    status = hs.status;
  } else if (hs.status == SCS_DIVERGED) {
    status = SCS_DIVERGED;
  } else if (o.stop_rule != SCS_STOP_EPOCHS && !hs.done) {
    status = SCS_NOT_CONVERGED;
  } else if (rank_def) {
    status = SCS_SKETCH_RANK_DEFICIENT;
  }
  if (o.epoch_ms) {
    for (int s = 0; s < S; ++s) {
      float ms = -1.f;
      if (s > last_epoch || !epoch_events || hipEventElapsedTime(&ms, ev_start, ev_epoch(s)) != hipSuccess) ms = -1.f;
      o.epoch_ms[s] = ms;
    }
  }
  if (report) {
    std::memset(report, 0, sizeof(*report));
    report->status = status;
    report->epochs = hs.epochs;
    report->k_used = k_used;
    report->steps = m;
    report->eta = hs.eta;
    report->beta_hat = hs.beta_sum / (double)n;  // (1/(n+d)) sum beta_i with beta_i = (n+d)/n ||a_i||^2
    report->objective = hs.obj;
    report->grad_norm = std::sqrt(hs.gnorm2);
    report->certificate = hs.cert;
    report->lam_top = hs.lam_top;
    report->backoffs = hs.backoffs;
    report->workgroups = W;
    report->wave_rows =
        a.wave_rows == kInnerLookahead ? kInnerLookahead : inner_layout_wave_rows(b, d, W, a.wave_rows);
    float t1 = 0, t2 = 0, t3 = 0;
    hipEventElapsedTime(&t1, ev_start, ev_sketch);
    hipEventElapsedTime(&t2, ev_sketch, ev_apply);
    hipEventElapsedTime(&t3, ev_apply, ev_end);
    report->ms_sketch = t1;
    report->ms_apply = t2;
    report->ms_solve = t3;
    if (o.timing) {
      // launches that did work: the inner loops of hs.epochs epochs and the gradient passes before them
      // (plus the final evaluation when every epoch ran)
      int ng = o.timing >= 2 ? std::min(S + 1, hs.epochs + 1) : 0, ni = hs.epochs;
      double sg = 0.0, si = 0.0;
      for (int s = 0; s < ng; ++s) {
        float ms = 0.f;
        hipEventElapsedTime(&ms, ev_g0(s), ev_g1(s));
        sg += ms;
      }
      for (int s = 0; s < ni; ++s) {
        float ms = 0.f;
        hipEventElapsedTime(&ms, ev_i0(s), ev_epoch(s));
        si += ms;
      }
      report->ms_grad = sg;
      report->ms_inner = si;
      report->n_grad = ng;
      report->n_inner = ni;
    }
  }
  return status;
}

int scs_svrg_solve(scs_ctx* ctx, const float* X, int64_t n, int64_t d, int64_t ldx, const float* y, double lambda,
                   int k, double eps, const scs_opts* opts, float* w_out, scs_report* report) {
  return svrg_solve_impl(ctx, X, n, d, ldx, y, lambda, k, eps, opts, w_out, report, false);
}

int scs_autotune(scs_ctx* ctx, const float* X, int64_t n, int64_t d, int64_t ldx, const float* y, double lambda,
                 int k, double eps, const scs_opts* base, scs_opts* tuned, double* best_ms_out) {
  if (!ctx || !y || !tuned) {
    set_error("autotune: null argument");
    return SCS_EINVAL;
  }
  SCS_CHECK(validate_problem(X, n, d, ldx, lambda));
  scs_opts o;
  scs_opts_default(&o);
  if (base) o = *base;
  if (o.omega || o.indices || o.trace_w || o.stop_rule == SCS_STOP_EPOCHS) {
    set_error("autotune: needs a stopping rule that ends the solve (certificate or gap) and no injected omega, "
              "indices or trace");
    return SCS_EINVAL;
  }
  o.epoch_ms = nullptr;
  o.timing = 0;
  o.steps = 0;
  o.workgroups = -1;  // every candidate's inner-loop shape is itself timed (cached per (d, b, precision))
  o.wave_rows = 0;
  o.seed = o.seed ^ 0x5ca1ab1e5eedull;  // candidates never see the caller's random streams
  Guard g(ctx->device);
  free_retired(ctx);
  WS(wt, float, "tune_w", (size_t)d);
  // warm-up: first-use workspace and the inner-loop shape for b = 64
  {
    scs_opts w0 = o;
    w0.max_epochs = 1;
    w0.stop_rule = SCS_STOP_EPOCHS;
    SCS_CHECK(svrg_solve_impl(ctx, X, n, d, ldx, y, lambda, k, eps, &w0, wt, nullptr, false));
  }
  const int bs[] = {32, 64, 128};
  const double mfs[] = {1.0 / 64, 1.0 / 32, 1.0 / 16, 1.0 / 8, 1.0 / 4, 1.0 / 2, 1.0, 2.0};
  const double cs[] = {1, 2, 4, 8, 16, 32, 64, 128, 256, 512};
  double best = 1e300;
  scs_opts best_o = o;
  bool found = false;
  std::vector<std::pair<double, scs_opts>> done;  // every candidate that reached the stopping rule
  for (int b : bs) {
    for (double mf : mfs) {
      if (mf * (double)n / b < 1.0) continue;
      int worse = 0;
      double best_here = 1e300;
      for (double c : cs) {
        scs_opts t = o;
        t.batch = b;
        t.epoch_factor = mf;
        t.step_scale = c;
        scs_report rep;
        const auto t0 = std::chrono::steady_clock::now();
        const int rc = svrg_solve_impl(ctx, X, n, d, ldx, y, lambda, k, eps, &t, wt, &rep, false);
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (rc < 0) return rc;
        if (rc == SCS_DIVERGED || rep.backoffs > 0) break;  // larger steps only diverge further
        if (rc == SCS_OK || rc == SCS_SKETCH_RANK_DEFICIENT) {
          t.workgroups = rep.workgroups;
          done.emplace_back(ms, t);
          if (ms < best) {
            best = ms;
            best_o = t;
            found = true;
          }
          if (ms < best_here) {
            best_here = ms;
            worse = 0;
          } else if (++worse >= 2) {
            break;  // past the best step of this (b, m): the time has risen twice in a row
          }
        }
      }
    }
  }
  if (!found) {
    set_error("autotune: no candidate reached the stopping rule within max_epochs");
    return SCS_NOT_CONVERGED;
  }
  // One timing per candidate ranks them only roughly: the epoch count a candidate needs moves by one
  // from one sampler stream to the next, and that step is a large share of a short solve. The fastest
  // few are timed again over further sampler streams and the lowest median wins.
  {
    constexpr int kFinalists = 4, kStreams = 4;
    std::stable_sort(done.begin(), done.end(),
                     [](const std::pair<double, scs_opts>& a, const std::pair<double, scs_opts>& b) {
                       return a.first < b.first;
                     });
    if (done.size() > (size_t)kFinalists) done.resize(kFinalists);
    double best_med = 1e300;
    for (auto& cand : done) {
      double ms_s[kStreams] = {cand.first};
      for (int r = 1; r < kStreams; ++r) {
        scs_opts t = cand.second;
        t.seed = o.seed ^ (0x9e3779b97f4a7c15ull * (uint64_t)r);
        t.workgroups = -1;  // the same cached shape as the first timing
        scs_report rep;
        const auto t0 = std::chrono::steady_clock::now();
        const int rc = svrg_solve_impl(ctx, X, n, d, ldx, y, lambda, k, eps, &t, wt, &rep, false);
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (rc < 0) return rc;
        ms_s[r] = (rc == SCS_OK || rc == SCS_SKETCH_RANK_DEFICIENT) && rep.backoffs == 0 ? ms : 1e300;
      }
      std::sort(ms_s, ms_s + kStreams);
      const double med = 0.5 * (ms_s[kStreams / 2 - 1] + ms_s[kStreams / 2]);
      if (med < best_med) {
        best_med = med;
        best_o = cand.second;
      }
    }
    best = best_med;
  }
  // the inner-loop shape the solves used (the context's cached choice for this b), then the caller's seed
  auto it = ctx->tuned_w.find(std::to_string(d) + "/" + std::to_string(best_o.batch) + "/" +
                              std::to_string(best_o.precision == SCS_PREC_MIXED ? 1 : 0));
  if (it != ctx->tuned_w.end()) {
    best_o.workgroups = it->second.first;
    best_o.wave_rows = it->second.second;
  }
  best_o.seed = base ? base->seed : o.seed ^ 0x5ca1ab1e5eedull;
  best_o.epoch_ms = base ? base->epoch_ms : nullptr;
  best_o.timing = base ? base->timing : 0;
  *tuned = best_o;
  if (best_ms_out) *best_ms_out = best;
  return SCS_OK;
}

// ================================================================ the FP64 path
// The one-block sketch (Alg. 2 with q = 1) of FP64 X, every product in FP64: T = X Omega, Y = X^T T,
// Q = CholeskyQR2(Y), W = X Q, B = W^T W / n = V Theta V^T, U~ = Q V_k, lam = Theta_{1..k}, and with
// want_z also Z = X U~ (n x k). Leaves f64_U (d x k), f64_lam (k) and f64_Z in the workspace; flags
// (device, 2 ints) receive CholeskyQR's breakdown flags. Omega^T is o.omega (FP32, l x d) or drawn
// from o.seed, as in the FP32 path, and widened to FP64.
static int sketch64_impl(scs_ctx* ctx, hipStream_t st, const double* X, int64_t n, int64_t d, int64_t ldx, int k,
                         const scs_opts& o, bool want_z, int* flags) {
  const int l = k + o.oversample;
  const float* om32 = o.omega;
  if (!om32) {
    WS(g32, float, "f64_omega32", (size_t)l * d);
    SCS_CHECK(launch_gaussian(st, o.seed, (int64_t)l * d, g32));
    om32 = g32;
  }
  WS(om, double, "f64_omega", (size_t)l * d);
  SCS_CHECK(launch_f32_to_f64(st, (int64_t)l * d, om32, om));
  WS(T, double, "f64_T", (size_t)n * l);
  WS(Y, double, "f64_Y", (size_t)d * l);
  SCS_CHECK(launch_gemm64(st, n, l, d, X, ldx, 1, om, 1, d, T, l, nullptr, 0));  // T = X Omega
  SCS_CHECK(launch_gemm64(st, d, l, n, X, 1, ldx, T, l, 1, Y, l, nullptr, 0));   // Y = X^T T
  WS(Rinv, double, "f64_Rinv", (size_t)l * l);
  WS(Q1, double, "f64_Q1", (size_t)d * l);
  WS(Q, double, "f64_Q", (size_t)d * l);
  WS(G, double, "f64_G", (size_t)l * l);
  WS(Rp, double, "f64_Rp", (size_t)l * (l + 1) / 2 + l);
  WS(Gp, double, "f64_Gpart", (size_t)gram64_parts(d) * l * l);
  WS(cgate, int, "f64_chol_gate", 1);
  SCS_CHECK(cholqr2_64(st, d, l, Y, Q, l, nullptr, flags, G, Rinv, Q1, Rp, Gp, cgate));
  // Rayleigh-Ritz: W = X Q (over T), B = W^T W / n
  SCS_CHECK(launch_gemm64(st, n, l, d, X, ldx, 1, Q, l, 1, T, l, nullptr, 0));
  WS(B, double, "f64_B", (size_t)l * l);
  SCS_CHECK(launch_gemm64(st, l, l, n, T, 1, l, T, l, 1, B, l, nullptr, 0));
  SCS_CHECK(launch_scale64(st, (int64_t)l * l, 1.0 / (double)n, B));
  WS(V, double, "f64_V", (size_t)l * l);
  WS(theta, double, "f64_theta", (size_t)l);
  WS(order, int, "f64_order", (size_t)l);
  WS(eigw, double, "f64_eig_work", eig64_work_len(l));
  SCS_CHECK(launch_eig64(st, B, l, eigw, V, theta, order));
  WS(U, double, "f64_U", (size_t)d * k);
  WS(lam, double, "f64_lam", (size_t)k);
  WS(U32, float, "f64_U32", (size_t)d * k);
  WS(UT32, float, "f64_UT32", (size_t)k * d);
  WS(VkT, float, "f64_VkT", (size_t)k * l);
  SCS_CHECK(launch_lift(st, Q, d, l, V, order, k, theta, U, U32, UT32, lam, VkT));
  if (want_z) {
    WS(Z, double, "f64_Z", (size_t)n * k);
    SCS_CHECK(launch_gemm64(st, n, k, d, X, ldx, 1, U, k, 1, Z, k, nullptr, 0));  // Z = X U~
  }
  return SCS_OK;
}

static int check_f64_problem(const double* X, int64_t n, int64_t d, int64_t ldx, double lambda, int k,
                             const scs_opts& o) {
  SCS_CHECK(validate_problem(X, n, d, ldx, lambda));
  if (d > kF64MaxD || n + d > INT32_MAX) {
    set_error("FP64 path: need d <= 4096 and n + d < 2^31");
    return SCS_EINVAL;
  }
  if (k < 0 || k > d || (k > 0 && (o.oversample < 0 || o.krylov_blocks > 1 || k + o.oversample > d ||
                                   k + o.oversample > n || k + o.oversample > kF64MaxL))) {
    set_error("FP64 path: need 0 <= k and, for k > 0, one Krylov block and k + p <= min(d, n, 136)");
    return SCS_EINVAL;
  }
  return SCS_OK;
}

static int svrg_solve_f64_impl(scs_ctx* ctx, const double* X, int64_t n, int64_t d, int64_t ldx, const double* y,
                               double lambda, int k, double eps, const scs_opts* opts, double* w_out,
                               scs_report* report, bool sketch_failed) {
  if (!ctx || !y || !w_out) {
    set_error("null argument");
    return SCS_EINVAL;
  }
  scs_opts o;
  scs_opts_default(&o);
  if (opts) o = *opts;
  SCS_CHECK(check_f64_problem(X, n, d, ldx, lambda, k, o));
  if (o.batch < 1 || o.batch > kInnerMaxB || o.max_epochs < 1 || o.steps < 0 || !(o.step_scale > 0.0) ||
      !(o.epoch_factor >= 0.0) || o.stop_rule < 0 || o.stop_rule > 2 || o.epoch_offset < 0 || o.w0 || o.trace_w ||
      o.wt_out) {
    set_error("FP64 path: need 1 <= batch <= 256, max_epochs >= 1, steps >= 0, step_scale > 0, epoch_offset >= 0; "
              "w0, trace_w and wt_out are FP32-only");
    return SCS_EINVAL;
  }
  Guard g(ctx->device);
  free_retired(ctx);
  hipStream_t st = ctx->stream;
  const int b = o.batch;
  const int64_t m = epoch_steps(o, n, b);
  const int64_t N = n + d;
  const int S = o.max_epochs;
  const int64_t ldt = cdiv(d, 32) * 32;  // rows start on 256-byte boundaries
  // events: 0 start, 1 sketch done, 2 rows and sampler done, 3 end, 4 + s end of epoch s; with timing,
  // 4 + S + s opens the inner loop of epoch s
  SCS_CHECK(ensure_events(ctx, 0, (size_t)(o.timing ? 4 + 2 * S : 4 + S)));
  SCS_CHECK(ensure_stop_flags(ctx, (size_t)S + 3));
  std::memset(ctx->stop_flags, 0, sizeof(int) * (S + 3));
  int* chol_flags = ctx->stop_flags + S + 1;
  hipEvent_t* tev = ctx->tevents.data();
  SCS_HIP(hipEventRecord(tev[0], st));
  WS(state, SolveState, "f64_state", 1);
  SCS_HIP(hipMemsetAsync(state, 0, sizeof(SolveState), st));

  // ---- sketch (Alg. 3's first step); a CholeskyQR breakdown reruns the solve with P = I
  const int k_used = sketch_failed ? 0 : k;
  if (k_used > 0) {
    SCS_CHECK(sketch64_impl(ctx, st, X, n, d, ldx, k, o, true, chol_flags));
    SCS_HIP(hipStreamSynchronize(st));
    if (__atomic_load_n(chol_flags, __ATOMIC_ACQUIRE) || __atomic_load_n(chol_flags + 1, __ATOMIC_ACQUIRE))
      return svrg_solve_f64_impl(ctx, X, n, d, ldx, y, lambda, k, eps, opts, w_out, report, true);
  }
  SCS_HIP(hipEventRecord(tev[1], st));

  // ---- preconditioned rows a_i (data, then regularizer) and beta_i = ||a_i||^2
  WS(Xt, double, "f64_Xt", (size_t)n * ldt);
  WS(reg, double, "f64_reg", (size_t)d * ldt);
  WS(beta, double, "f64_beta", (size_t)N);
  const double* U = nullptr;
  const double* lam = nullptr;
  const double* UT = nullptr;
  const double sq = std::sqrt((double)n * lambda);
  if (k_used > 0) {
    U = ws<double>(ctx, "f64_U", 0);
    lam = ws<double>(ctx, "f64_lam", 0);
    WS(UTb, double, "f64_UT", (size_t)k_used * d);
    WS(UDT, double, "f64_UDT", (size_t)k_used * d);
    SCS_CHECK(launch_precond_setup64(st, U, lam, k_used, d, lambda, UTb, UDT, state));
    SCS_CHECK(launch_rows64(st, n, ws<double>(ctx, "f64_Z", 0), k_used, UDT, k_used, X, ldx, d, lam, lambda, 1.0, Xt,
                            ldt, beta));
    SCS_CHECK(launch_rows64(st, d, U, k_used, UDT, k_used, nullptr, 0, d, lam, lambda, sq, reg, ldt, beta + n));
    UT = UTb;
  } else {
    SCS_CHECK(launch_rows64(st, n, nullptr, 0, nullptr, 0, X, ldx, d, nullptr, lambda, 1.0, Xt, ldt, beta));
    SCS_CHECK(launch_rows64(st, d, nullptr, 0, nullptr, 0, nullptr, 0, d, nullptr, lambda, sq, reg, ldt, beta + n));
  }
  // ---- sampling weights (Alg. 1: q_i = beta_i / sum beta)
  WS(cum, uint64_t, "f64_cum", (size_t)N);
  WS(scr, double, "f64_sampler_scratch", (size_t)sampler_scratch_len(N));
  SCS_CHECK(launch_sampler_prepare(st, beta, N, cum, scr, sampler_scratch_len(N), state, o.uniform_sampling));
  SCS_HIP(hipEventRecord(tev[2], st));

  // ---- SVRG epochs (Alg. 1)
  const int nwg = grad64_workgroups(n);
  WS(wt, double, "f64_wt", (size_t)d);
  WS(wt_prev, double, "f64_wt_prev", (size_t)d);
  WS(w, double, "f64_w", (size_t)d);
  WS(mu, double, "f64_mu", (size_t)d);
  WS(part, double, "f64_gpart", (size_t)nwg * d);
  WS(rsq, double, "f64_grsq", (size_t)nwg);
  constexpr int kSampleGroup = 8;  // epochs of index draws per sampler launch
  WS(idxb, int32_t, "f64_idx", (size_t)kSampleGroup * m * b);
  WS(scale, double, "f64_scale", (size_t)kSampleGroup * m * b);
  SCS_CHECK(launch_zero3(st, wt, (int64_t)sizeof(double) * d, wt_prev, (int64_t)sizeof(double) * d, nullptr, 0));
  Inner64Args a{};
  a.n = n;
  a.d = d;
  a.Xt = Xt;
  a.reg = reg;
  a.ld = ldt;
  a.m = m;
  a.b = b;
  a.mu = mu;
  a.wt = wt;
  a.wt_prev = wt_prev;
  a.step_scale = o.step_scale;
  a.average = o.average;
  a.state = state;
  constexpr int kLookahead = 3;
  int last_epoch = -1;
  const bool epoch_events = o.epoch_ms != nullptr || o.timing != 0;  // as in the FP32 solve
  for (int s = 0; s <= S; ++s) {
    SCS_CHECK(launch_premap64(st, UT, lam, k_used, d, lambda, wt, w, state));
    SCS_CHECK(launch_grad64(st, X, n, d, ldx, y, w, nwg, part, rsq, state));
    SCS_CHECK(launch_finish64(st, part, rsq, nwg, n, d, w, lambda, UT, lam, k_used, mu, state, o.stop_rule, eps,
                              o.f_star, wt, wt_prev, s == 0 ? 1 : 0, ctx->stop_flags + s));
    if (s == S) break;
    const int64_t mb = m * b, slot = s % kSampleGroup;
    if (slot == 0) {
      const int64_t cnt = (int64_t)std::min(kSampleGroup, S - s) * mb;
      if (o.indices) SCS_CHECK(launch_index_scale(st, cum, N, n, o.indices + (int64_t)s * mb, cnt, scale, state));
      else SCS_CHECK(launch_sample(st, cum, N, n, o.seed, s + o.epoch_offset, mb, cnt, idxb, scale, state));
    }
    a.idx = o.indices ? o.indices + (int64_t)s * mb : idxb + slot * mb;
    a.scale = scale + slot * mb;
    if (o.timing) SCS_HIP(hipEventRecord(tev[4 + S + s], st));
    SCS_CHECK(launch_inner64(st, a));
    if (epoch_events) SCS_HIP(hipEventRecord(tev[4 + s], st));
    last_epoch = s;
    if (s + 1 >= kLookahead) {  // as in the FP32 solve: stop enqueuing once a finished snapshot is seen
      const int q = s + 1 - kLookahead;
      int flag = 0;
      SCS_CHECK(wait_stop_flag(ctx, st, q, &flag));
      if (flag == 1) break;
    }
  }
  SCS_CHECK(launch_premap64(st, UT, lam, k_used, d, lambda, wt, w_out, nullptr));
  SCS_HIP(hipEventRecord(tev[3], st));
  SolveState hs;
  SCS_HIP(hipMemcpyAsync(&hs, state, sizeof(hs), hipMemcpyDeviceToHost, st));
  SCS_HIP(hipStreamSynchronize(st));

  int status = SCS_OK;
  if (hs.status == SCS_ENONFINITE) {
    set_error("non-finite value in X or y");
    status = hs.status;
  } else if (hs.status == SCS_DIVERGED) {
    status = SCS_DIVERGED;
  } else if (o.stop_rule != SCS_STOP_EPOCHS && !hs.done) {
    status = SCS_NOT_CONVERGED;
  } else if (sketch_failed) {
    status = SCS_SKETCH_RANK_DEFICIENT;
  }
  if (o.epoch_ms) {
    for (int s = 0; s < S; ++s) {
      float ms = -1.f;
      if (s > last_epoch || !epoch_events || hipEventElapsedTime(&ms, tev[0], tev[4 + s]) != hipSuccess) ms = -1.f;
      o.epoch_ms[s] = ms;
    }
  }
  if (report) {
    std::memset(report, 0, sizeof(*report));
    report->status = status;
    report->epochs = hs.epochs;
    report->k_used = k_used;
    report->steps = m;
    report->eta = hs.eta;
    report->beta_hat = hs.beta_sum / (double)n;
    report->objective = hs.obj;
    report->grad_norm = std::sqrt(hs.gnorm2);
    report->certificate = hs.cert;
    report->lam_top = hs.lam_top;
    report->backoffs = hs.backoffs;
    report->workgroups = 1;
    report->wave_rows = 0;
    float t1 = 0, t2 = 0, t3 = 0;
    hipEventElapsedTime(&t1, tev[0], tev[1]);
    hipEventElapsedTime(&t2, tev[1], tev[2]);
    hipEventElapsedTime(&t3, tev[2], tev[3]);
    report->ms_sketch = t1;
    report->ms_apply = t2;
    report->ms_solve = t3;
    if (o.timing) {
      double si = 0.0;
      for (int s = 0; s < hs.epochs; ++s) {
        float ms = 0.f;
        hipEventElapsedTime(&ms, tev[4 + S + s], tev[4 + s]);
        si += ms;
      }
      report->ms_inner = si;
      report->n_inner = hs.epochs;
    }
  }
  return status;
}

int scs_sketch_build_f64(scs_ctx* ctx, const double* X, int64_t n, int64_t d, int64_t ldx, int k,
                         const scs_opts* opts, double* U_out, double* lam_out) {
  if (!ctx || !U_out || !lam_out) {
    set_error("null argument");
    return SCS_EINVAL;
  }
  scs_opts o;
  scs_opts_default(&o);
  if (opts) o = *opts;
  SCS_CHECK(check_f64_problem(X, n, d, ldx, 1.0, k, o));
  if (k < 1) {
    set_error("sketch: need k >= 1");
    return SCS_EINVAL;
  }
  Guard g(ctx->device);
  free_retired(ctx);
  hipStream_t st = ctx->stream;
  int* flags = ws<int>(ctx, "f64_cholflags", 2);
  if (!flags) return SCS_ENOMEM;
  SCS_CHECK(sketch64_impl(ctx, st, X, n, d, ldx, k, o, false, flags));
  SCS_HIP(hipMemcpyAsync(U_out, ws<double>(ctx, "f64_U", 0), sizeof(double) * d * k, hipMemcpyDeviceToDevice, st));
  SCS_HIP(hipMemcpyAsync(lam_out, ws<double>(ctx, "f64_lam", 0), sizeof(double) * k, hipMemcpyDeviceToDevice, st));
  int hflags[2] = {0, 0};
  SCS_HIP(hipMemcpyAsync(hflags, flags, sizeof(hflags), hipMemcpyDeviceToHost, st));
  SCS_HIP(hipStreamSynchronize(st));
  return hflags[0] || hflags[1] ? SCS_SKETCH_RANK_DEFICIENT : SCS_OK;
}

int scs_svrg_solve_f64(scs_ctx* ctx, const double* X, int64_t n, int64_t d, int64_t ldx, const double* y,
                       double lambda, int k, double eps, const scs_opts* opts, double* w_out, scs_report* report) {
  return svrg_solve_f64_impl(ctx, X, n, d, ldx, y, lambda, k, eps, opts, w_out, report, false);
}

int scs_svrg_solve_batched(scs_ctx* ctx, int nprob, const float* const* X, const int64_t* n, const int64_t* d,
                           const int64_t* ldx, const float* const* y, const double* lambda, const int* k, double eps,
                           const double* f_star, const scs_opts* opts, float* const* w_out, scs_report* reports) {
  if (!ctx || nprob < 1 || !X || !n || !d || !ldx || !y || !lambda || !k || !w_out) {
    set_error("null argument or nprob < 1");
    return SCS_EINVAL;
  }
  scs_opts o;
  scs_opts_default(&o);
  if (opts) o = *opts;
  if (o.omega || o.indices || o.trace_w || o.w0 || o.wt_out || o.epoch_offset != 0 || o.warm_start) {
    set_error("batched solve: omega, indices, trace_w, w0, wt_out must be NULL, epoch_offset and warm_start 0");
    return SCS_EINVAL;
  }
  if (o.stop_rule == SCS_STOP_GAP && !f_star) {
    set_error("batched solve: the gap rule needs f_star, one optimum per problem");
    return SCS_EINVAL;
  }
  if (o.batch < 1 || o.batch > kInnerMaxB || o.max_epochs < 1 || o.steps < 0 || !(o.step_scale > 0.0) ||
      !(o.epoch_factor >= 0.0) || o.stop_rule < 0 || o.stop_rule > 2) {
    set_error("bad options: need 1 <= batch <= 256, max_epochs >= 1, steps >= 0, step_scale > 0");
    return SCS_EINVAL;
  }
  int64_t max_d = 0;
  std::vector<int> vec4(nprob);
  for (int p = 0; p < nprob; ++p) {
    SCS_CHECK(validate_problem(X[p], n[p], d[p], ldx[p], lambda[p]));
    const int l = k[p] + o.oversample;
    if (!y[p] || !w_out[p] || k[p] < 0 || k[p] > d[p] ||
        (k[p] > 0 && (o.oversample < 0 || !sketch_width_ok(o, k[p], n[p], d[p]))) || n[p] + d[p] > INT32_MAX) {
      set_error("batched solve: problem " + std::to_string(p) +
                ": need y, w_out, 0 <= k and, for k > 0, q (k + p) <= min(d, n, 136) for q Krylov blocks");
      return SCS_EINVAL;
    }
    max_d = std::max(max_d, d[p]);
    vec4[p] = d[p] % 4 == 0 && ldx[p] % 4 == 0 && (uintptr_t)X[p] % 16 == 0;
  }
  // kernel order: problems whose rows allow float4 loads first, so each row layout of the gradient
  // pass gets one launch over a contiguous range (the layout a single solve would use)
  std::vector<int> kord;
  for (int p = 0; p < nprob; ++p)
    if (vec4[p]) kord.push_back(p);
  const int nv = (int)kord.size();
  for (int p = 0; p < nprob; ++p)
    if (!vec4[p]) kord.push_back(p);
  // largest first inside each group (when the inner loop needs several launches, the longest
  // problems start first)
  auto bigger = [&](int a_, int b_) { return n[a_] * d[a_] > n[b_] * d[b_]; };
  std::stable_sort(kord.begin(), kord.begin() + nv, bigger);
  std::stable_sort(kord.begin() + nv, kord.end(), bigger);
  std::vector<int> sidx(nprob);
  for (int i = 0; i < nprob; ++i) sidx[kord[i]] = i;
  if (max_d > 16 * batched_max_slice(o.batch)) {
    set_error("batched solve: d > 8192 (2048 for batch > 64, 1024 for batch > 128)");
    return SCS_EINVAL;
  }
  Guard g(ctx->device);
  free_retired(ctx);
  hipStream_t st = ctx->stream;
  const int b = o.batch, S = o.max_epochs, mixed = o.precision == SCS_PREC_MIXED;
  const int es = mixed ? 2 : 4;
  constexpr int G = 8;  // epochs of index streams drawn per sampling launch
  // W cooperating workgroups per problem (the same for every problem of the batch): opts.workgroups
  // when positive, else one per 256 columns of the widest problem (measured: 256-column slices beat
  // both 512 and 128 on the uneven batch); a slice never exceeds 512 columns
  const int64_t maxs = batched_max_slice(o.batch);
  const int W = (int)std::min<int64_t>(
      16, std::max<int64_t>(cdiv(max_d, maxs),
                            o.workgroups > 0 ? (int64_t)o.workgroups : cdiv(max_d, std::min<int64_t>(256, maxs))));

  // ---- per-problem sizes and arena offsets (elements)
  std::vector<int64_t> ldt(nprob), m(nprob), nwg(nprob), o_xt(nprob), o_reg(nprob), o_beta(nprob), o_vec(nprob),
      o_g64(nprob), o_gp(nprob), o_gr(nprob), o_idx(nprob), o_ut(nprob), o_lam(nprob);
  int64_t t_xt = 0, t_reg = 0, t_beta = 0, t_vec = 0, t_g64 = 0, t_gp = 0, t_gr = 0, t_idx = 0, t_ut = 0, t_lam = 0;
  int64_t max_N = 0;
  for (int p = 0; p < nprob; ++p) {
    ldt[p] = cdiv(d[p], mixed ? 128 : 64) * (mixed ? 128 : 64);
    m[p] = epoch_steps(o, n[p], b);
    nwg[p] = grad_num_workgroups(n[p], d[p]);  // as in a single solve, so the sums agree bit for bit
    o_xt[p] = t_xt;
    t_xt += n[p] * ldt[p];
    o_reg[p] = t_reg;
    t_reg += d[p] * ldt[p];
    o_beta[p] = t_beta;
    t_beta += n[p] + d[p];
    o_vec[p] = t_vec;
    t_vec += d[p];
    o_g64[p] = t_g64;
    t_g64 += 16 * d[p];
    o_gp[p] = t_gp;
    t_gp += nwg[p] * d[p];
    o_gr[p] = t_gr;
    t_gr += nwg[p];
    o_idx[p] = t_idx;
    t_idx += (int64_t)G * m[p] * b;
    o_ut[p] = t_ut;
    t_ut += cdiv((int64_t)k[p] * d[p], 4) * 4;  // 16-byte aligned blocks
    o_lam[p] = t_lam;
    t_lam += k[p];
    max_N = std::max(max_N, n[p] + d[p]);
  }
  void* xt_all = wsb(ctx, "b_xt", (size_t)t_xt * es);
  void* reg_all = wsb(ctx, "b_reg", (size_t)t_reg * es);
  if (!xt_all || !reg_all) return SCS_ENOMEM;
  WS(beta_all, float, "b_beta", t_beta);
  WS(cum_all, uint64_t, "b_cum", t_beta);
  WS(vec_all, float, "b_vec", 4 * t_vec);  // wt | wt_prev | w32 | mu
  WS(tmp_all, double, "b_tmp", t_vec);
  WS(g64_all, double, "b_g64", t_g64);
  WS(gp_all, float, "b_gpart", t_gp);
  WS(gr_all, double, "b_grsq", t_gr);
  WS(idx_all, int32_t, "b_idx", t_idx);
  WS(sc_all, float, "b_scale", t_idx);
  WS(ut_all, float, "b_UT", std::max<int64_t>(t_ut, 1));
  WS(lam_all, double, "b_lam", std::max<int64_t>(t_lam, 1));
  WS(xbuf_all, uint64_t, "b_xbuf", (int64_t)nprob * inner_xbuf_words(W));
  WS(states, SolveState, "b_state", nprob);
  WS(flags_all, int, "b_cholflags", 2 * nprob);
  WS(gates_all, int, "b_cholgates", nprob);  // written by the batched CholeskyQR2 before it reads them
  WS(done_count, int, "b_done", 1);
  WS(desc, BatchProb, "b_desc", nprob);
  WS(prefix, int64_t, "b_prefix", 3 * ((int64_t)nprob + 1));
  WS(wout_dev, float*, "b_wout", nprob);
  WS(scr, double, "sampler_scratch", (size_t)sampler_scratch_len(max_N));
  SCS_HIP(hipMemsetAsync(states, 0, sizeof(SolveState) * nprob, st));
  SCS_HIP(hipMemsetAsync(vec_all, 0, sizeof(float) * 2 * t_vec, st));  // wt and wt_prev start at 0
  SCS_HIP(hipMemsetAsync(xbuf_all, 0, sizeof(uint64_t) * nprob * inner_xbuf_words(W), st));
  SCS_HIP(hipMemsetAsync(flags_all, 0, sizeof(int) * 2 * nprob, st));
  SCS_HIP(hipMemsetAsync(done_count, 0, sizeof(int), st));

  // tev: 0 start, 1-2 stage ends, 3 end, 4 + s end of epoch s (where the host reads stop flag s);
  // with timing, 4 + S + s opens the inner loop of epoch s
  SCS_CHECK(ensure_events(ctx, 0, (size_t)4 + (o.timing ? 2 * S : S)));
  SCS_CHECK(ensure_stop_flags(ctx, (size_t)S + 1));
  std::memset(ctx->stop_flags, 0, sizeof(int) * (S + 1));
  hipEvent_t* tev = ctx->tevents.data();
  SCS_HIP(hipEventRecord(tev[0], st));

  // ---- per-problem setup (largest first, so shared sketch temporaries are sized once)
  std::vector<int> ord(nprob);
  for (int p = 0; p < nprob; ++p) ord[p] = p;
  std::stable_sort(ord.begin(), ord.end(), [&](int a_, int b_) { return n[a_] * d[a_] > n[b_] * d[b_]; });
  auto setup_identity = [&](int p, hipStream_t sq, const std::string& sfx) -> int {
    char* xt = (char*)xt_all + o_xt[p] * es;
    char* rg = (char*)reg_all + o_reg[p] * es;
    float* beta = beta_all + o_beta[p];
    if (mixed) {
      WS(tmp16, uint16_t, "xcopy16" + sfx, n[p] * d[p]);
      SCS_CHECK(launch_copy_bf16(sq, X[p], n[p], d[p], ldx[p], tmp16));
      SCS_HIP(hipMemcpy2DAsync(xt, ldt[p] * 2, tmp16, d[p] * 2, d[p] * 2, n[p], hipMemcpyDeviceToDevice, sq));
      SCS_CHECK(launch_rownorm_bf16(sq, tmp16, n[p], d[p], beta));
    } else {
      SCS_HIP(hipMemcpy2DAsync(xt, ldt[p] * 4, X[p], ldx[p] * 4, d[p] * 4, n[p], hipMemcpyDeviceToDevice, sq));
      SCS_CHECK(launch_rownorm(sq, X[p], n[p], d[p], ldx[p], beta));
    }
    WS(rtmp, float, "regtmp" + sfx, d[p] * d[p]);
    SCS_CHECK(launch_fill_scaled_identity(sq, d[p], std::sqrt((double)n[p] * lambda[p]), mixed, rtmp, beta + n[p]));
    SCS_HIP(hipMemcpy2DAsync(rg, ldt[p] * es, rtmp, d[p] * es, d[p] * es, d[p], hipMemcpyDeviceToDevice, sq));
    return SCS_OK;
  };
  // Problems are independent until their epochs: their sketches, preconditioned rows and sampling
  // weights are built on up to kLanes streams at once (each with its own workspace buffers), largest
  // problems first, so the latency-bound small kernels of different problems overlap on different
  // CUs. (256 uneven problems: 16 lanes 40.5 ms, 8 lanes 46.3 ms; the runtime's 4 hardware queues
  // are shared by the lanes, and 16 or 32 queues gave no gain.)
  constexpr int kLanes = 16;
  const int lanes = std::min(nprob, kLanes);
  SCS_CHECK(ensure_side_streams(ctx, lanes));
  SCS_HIP(hipEventRecord(tev[1], st));
  for (int q = 0; q < lanes; ++q) SCS_HIP(hipStreamWaitEvent(ctx->side[q], tev[1], 0));
  // Five phases. 1 (lanes): each problem's range finder Y = X^T (X Omega), kept in a buffer of its own.
  // 2 (one stream): CholeskyQR2 of every Y, eleven launches for all problems. 3 (lanes): X Q and the
  // Rayleigh-Ritz matrix B, kept with Q and X Q. 4 (one stream): the eigendecompositions of every B
  // and the lifts U~ = Q V_k, one launch each for all problems (one workgroup per problem), writing
  // U~^T and lam~ straight into the batch arrays. 5 (lanes): Z = (X Q) V_k, the preconditioned rows
  // and the sampling weights. Problems without a sketch are set up in phase 1; with several Krylov
  // blocks (CholeskyQR2 once per block, between the block's GEMMs) a sketch runs whole in phase 1.
  auto join_lanes = [&]() -> int {
    for (int q = 0; q < lanes; ++q) {
      SCS_HIP(hipEventRecord(ctx->side_events[q], ctx->side[q]));
      SCS_HIP(hipStreamWaitEvent(st, ctx->side_events[q], 0));
    }
    return SCS_OK;
  };
  auto prepare_sampler = [&](int p, hipStream_t sq, const std::string& sfx) -> int {
    // with the lane's own scratch (a problem whose CholeskyQR breaks down is redone below)
    WS(lscr, double, "sampler_scratch" + sfx, (size_t)sampler_scratch_len(max_N));
    return launch_sampler_prepare(sq, beta_all + o_beta[p], n[p] + d[p], cum_all + o_beta[p], lscr,
                                  sampler_scratch_len(max_N), states + sidx[p], o.uniform_sampling);
  };
  std::vector<SketchSplit> split(nprob);
  const bool staged = std::max(1, o.krylov_blocks) == 1;
  for (int i = 0; i < nprob; ++i) {
    const int p = ord[i], lane = i % lanes;
    hipStream_t sq = ctx->side[lane];
    const std::string sfx = "#" + std::to_string(lane);
    if (k[p] > 0) {
      bool unused = false;
      split[p].stage = staged ? 1 : 0;
      SCS_CHECK(sketch_impl(ctx, X[p], n[p], d[p], ldx[p], k[p], o, true, &unused, flags_all + 2 * p, sq, sfx,
                            nullptr, &split[p], "#p" + std::to_string(p)));
    } else {
      SCS_CHECK(setup_identity(p, sq, sfx));
      SCS_CHECK(prepare_sampler(p, sq, sfx));
    }
  }
  SCS_CHECK(join_lanes());
  if (staged) {
    std::vector<CholJob> cj;
    int64_t max_dc = 1;
    int max_lc = 1;
    for (int p = 0; p < nprob; ++p) {
      if (k[p] <= 0) continue;
      const int l = split[p].l;
      const std::string ps = "#p" + std::to_string(p);
      WS(Gp, double, "Gpart64" + ps, (size_t)gram64_parts(d[p]) * l * l);
      WS(G, double, "G64" + ps, (size_t)l * l);
      WS(Rp, double, "Rp64" + ps, (size_t)l * (l + 1) / 2 + l);
      WS(Rinv, double, "Rinv64" + ps, (size_t)l * l);
      WS(Q1, double, "Q1_64" + ps, (size_t)d[p] * l);
      WS(Q, double, "Q64" + ps, (size_t)d[p] * l);
      WS(QT, float, "QT32" + ps, (size_t)l * d[p]);
      cj.push_back(CholJob{split[p].Y, d[p], l, Gp, G, Rp, Rinv, Q1, Q, l, QT, flags_all + 2 * p, gates_all + p});
      max_dc = std::max<int64_t>(max_dc, d[p]);
      max_lc = std::max(max_lc, l);
    }
    if (!cj.empty()) {
      WS(cjd, CholJob, "b_choljobs", cj.size());
      SCS_HIP(hipMemcpyAsync(cjd, cj.data(), sizeof(CholJob) * cj.size(), hipMemcpyHostToDevice, st));
      SCS_CHECK(launch_cholqr2_batched(st, cjd, (int)cj.size(), max_dc, max_lc));
      SCS_HIP(hipEventRecord(tev[2], st));
      for (int q = 0; q < lanes; ++q) SCS_HIP(hipStreamWaitEvent(ctx->side[q], tev[2], 0));
      for (int i = 0; i < nprob; ++i) {
        const int p = ord[i], lane = i % lanes;
        if (k[p] <= 0) continue;
        bool unused = false;
        split[p].stage = 2;
        SCS_CHECK(sketch_impl(ctx, X[p], n[p], d[p], ldx[p], k[p], o, true, &unused, flags_all + 2 * p,
                              ctx->side[lane], "#" + std::to_string(lane), nullptr, &split[p],
                              "#p" + std::to_string(p)));
      }
      SCS_CHECK(join_lanes());
    }
  }
  std::vector<Eig64Job> ej;
  std::vector<LiftJob> lj;
  std::vector<int> jp;  // problem of each job
  int max_L = 1;
  int64_t max_elems = 1;
  for (int p = 0; p < nprob; ++p) {
    if (k[p] <= 0) continue;
    const int L = split[p].L;
    const std::string ps = "#p" + std::to_string(p);
    WS(V, double, "V64" + ps, (size_t)L * L);
    WS(theta, double, "theta" + ps, (size_t)L);
    WS(order, int, "order" + ps, (size_t)L);
    WS(eigw, double, "eig_work" + ps, eig64_work_len(L));
    WS(U32, float, "U32" + ps, (size_t)d[p] * k[p]);
    WS(VkT, float, "VkT" + ps, (size_t)k[p] * L);
    ej.push_back(Eig64Job{split[p].B, L, eigw, V, theta, order});
    lj.push_back(LiftJob{split[p].Q, d[p], L, V, order, k[p], theta, nullptr, U32, ut_all + o_ut[p],
                         lam_all + o_lam[p], VkT});
    jp.push_back(p);
    max_L = std::max(max_L, L);
    max_elems = std::max(max_elems, std::max<int64_t>(d[p] * k[p], (int64_t)k[p] * L));
  }
  if (!ej.empty()) {
    WS(ejd, Eig64Job, "b_eigjobs", ej.size());
    WS(ljd, LiftJob, "b_liftjobs", lj.size());
    SCS_HIP(hipMemcpyAsync(ejd, ej.data(), sizeof(Eig64Job) * ej.size(), hipMemcpyHostToDevice, st));
    SCS_HIP(hipMemcpyAsync(ljd, lj.data(), sizeof(LiftJob) * lj.size(), hipMemcpyHostToDevice, st));
    SCS_CHECK(launch_eig64_batched(st, ejd, (int)ej.size(), max_L));
    SCS_CHECK(launch_lift_batched(st, ljd, (int)lj.size(), max_elems));
    SCS_HIP(hipEventRecord(tev[2], st));
    for (int q = 0; q < lanes; ++q) SCS_HIP(hipStreamWaitEvent(ctx->side[q], tev[2], 0));
    const int bf = mixed;
    for (size_t i = 0; i < jp.size(); ++i) {
      const int p = jp[i], lane = (int)(i % lanes);
      hipStream_t sq = ctx->side[lane];
      const std::string sfx = "#" + std::to_string(lane);
      const int64_t kz = gemm_wide_kpad(k[p]);
      WS(Z, float, "Z" + sfx, (size_t)n[p] * kz);
      SCS_CHECK(launch_gemm_nt_longk(sq, bf, split[p].Wq, n[p], split[p].L, split[p].Lp, lj[i].VkT, k[p],
                                     split[p].L, Z, kz, true));
      SCS_CHECK(apply_impl(ctx, X[p], n[p], d[p], ldx[p], lj[i].U32, Z, lam_all + o_lam[p], k[p], lambda[p], mixed,
                           mixed, (char*)xt_all + o_xt[p] * es, (char*)reg_all + o_reg[p] * es, ldt[p],
                           beta_all + o_beta[p], states + sidx[p], sq, sfx));
      SCS_CHECK(prepare_sampler(p, sq, sfx));
    }
    SCS_CHECK(join_lanes());
  }
  // CholeskyQR breakdown: those problems fall back to P = I (status SKETCH_RANK_DEFICIENT)
  std::vector<int> hflags(2 * nprob, 0);
  SCS_HIP(hipMemcpyAsync(hflags.data(), flags_all, sizeof(int) * 2 * nprob, hipMemcpyDeviceToHost, st));
  SCS_HIP(hipStreamSynchronize(st));
  std::vector<int> k_used(nprob), rank_def(nprob, 0);
  for (int p = 0; p < nprob; ++p) {
    k_used[p] = k[p];
    if (k[p] > 0 && (hflags[2 * p] || hflags[2 * p + 1])) {
      rank_def[p] = 1;
      k_used[p] = 0;
      SCS_CHECK(setup_identity(p, st, ""));
      SCS_CHECK(launch_sampler_prepare(st, beta_all + o_beta[p], n[p] + d[p], cum_all + o_beta[p], scr,
                                       sampler_scratch_len(max_N), states + sidx[p], o.uniform_sampling));
    }
  }
  SCS_HIP(hipEventRecord(tev[1], st));

  // ---- descriptors and flattened-grid prefixes
  std::vector<BatchProb> hp(nprob);
  std::vector<int64_t> pre(3 * ((size_t)nprob + 1), 0);
  int64_t* wg_pre = pre.data();
  int64_t* cb_pre = wg_pre + nprob + 1;
  int64_t* dr_pre = cb_pre + nprob + 1;
  int64_t max_slice = 0, max_d_v = 0, max_d_s = 0;
  std::vector<float*> wout_k(nprob);
  for (int i = 0; i < nprob; ++i) {
    const int p = kord[i];
    BatchProb& q = hp[i];
    wout_k[i] = w_out[p];
    (i < nv ? max_d_v : max_d_s) = std::max(i < nv ? max_d_v : max_d_s, d[p]);
    std::memset(&q, 0, sizeof(q));
    q.X = X[p];
    q.n = n[p];
    q.d = d[p];
    q.ldx = ldx[p];
    q.y = y[p];
    q.lambda = lambda[p];
    q.k = k_used[p];
    q.UT = k_used[p] > 0 ? ut_all + o_ut[p] : nullptr;
    q.lam = k_used[p] > 0 ? lam_all + o_lam[p] : nullptr;
    q.wt = vec_all + o_vec[p];
    q.wt_prev = vec_all + t_vec + o_vec[p];
    q.w32 = vec_all + 2 * t_vec + o_vec[p];
    q.mu = vec_all + 3 * t_vec + o_vec[p];
    q.tmp = tmp_all + o_vec[p];
    q.state = states + i;
    q.gpart = gp_all + o_gp[p];
    q.grsq = gr_all + o_gr[p];
    q.g64 = g64_all + o_g64[p];
    q.grows = 16;
    q.nwg = (int)nwg[p];
    q.stop_rule = o.stop_rule;
    q.eps = eps;
    q.f_star = f_star ? f_star[p] : 0.0;
    q.cum = cum_all + o_beta[p];
    q.N = n[p] + d[p];
    q.draws = m[p] * b;
    q.idx = idx_all + o_idx[p];
    q.scale = sc_all + o_idx[p];
    InnerArgs& a = q.inner;
    a.n = n[p];
    a.d = d[p];
    a.Xt = (char*)xt_all + o_xt[p] * es;
    a.ldx = ldt[p];
    a.reg = (char*)reg_all + o_reg[p] * es;
    a.ldr = ldt[p];
    a.mu = q.mu;
    a.m = m[p];
    a.b = b;
    a.eta_from_state = 1;
    a.step_scale = o.step_scale;
    a.average = o.average;
    a.W = W;
    a.xcd_stride = 1;
    a.slice = cdiv(cdiv(d[p], W), 4) * 4;
    a.wt = q.wt;
    a.wt_prev = q.wt_prev;
    a.xbuf = xbuf_all + (int64_t)p * inner_xbuf_words(W);
    a.state = q.state;
    max_slice = std::max(max_slice, a.slice);
    wg_pre[i + 1] = wg_pre[i] + nwg[p];
    cb_pre[i + 1] = cb_pre[i] + cdiv(d[p], 64);
    dr_pre[i + 1] = dr_pre[i] + (int64_t)G * m[p] * b;
  }
  if (max_slice > 512) {
    set_error("batched solve: column slice too wide");
    return SCS_EINVAL;
  }
  SCS_HIP(hipMemcpyAsync(desc, hp.data(), sizeof(BatchProb) * nprob, hipMemcpyHostToDevice, st));
  SCS_HIP(hipMemcpyAsync(prefix, pre.data(), sizeof(int64_t) * pre.size(), hipMemcpyHostToDevice, st));
  SCS_HIP(hipMemcpyAsync(wout_dev, wout_k.data(), sizeof(float*) * nprob, hipMemcpyHostToDevice, st));
  const int64_t* d_wg = prefix;
  const int64_t* d_cb = prefix + nprob + 1;
  const int64_t* d_dr = prefix + 2 * (nprob + 1);

  // ---- epochs of all problems in shared launches (Alg. 1 per problem)
  // One epoch of every problem; clk != nullptr: the epoch number comes from the device clock (graph replay).
  auto epoch_launches = [&](hipStream_t q, int s, const int* clk) -> int {
    SCS_CHECK(launch_premap_batched(q, desc, nprob, 0, nullptr));
    SCS_CHECK(launch_grad_partial_batched(q, desc, nprob, d_wg, 0, wg_pre[nv], max_d_v, 1));
    SCS_CHECK(launch_grad_partial_batched(q, desc, nprob, d_wg, wg_pre[nv], wg_pre[nprob] - wg_pre[nv], max_d_s, 0));
    SCS_CHECK(launch_grad_finish_batched(q, desc, nprob, d_cb, cb_pre[nprob], s == 0 ? 1 : 0, done_count,
                                         clk ? ctx->stop_flags : ctx->stop_flags + s, clk));
    if (!clk && s == S) return SCS_OK;
    const int slot = s % G;
    if (clk || slot == 0) SCS_CHECK(launch_sample_batched(q, desc, nprob, d_dr, dr_pre[nprob], o.seed, s, G, clk));
    if (o.timing) SCS_HIP(hipEventRecord(tev[4 + S + s], q));
    SCS_CHECK(launch_inner_epoch_batched(q, desc, nprob, W, max_slice, b, mixed, slot, s, clk));
    if (clk) SCS_CHECK(launch_clock_advance(q, ctx_clock(ctx)));
    return SCS_OK;
  };
  int epochs_launched = 0;
  int s0 = 0;
  bool stopped = false;
  if (!o.no_graph && !o.timing) SCS_CHECK(run_epoch_graph(ctx, st, S, epoch_launches, &s0, &stopped));
  constexpr int kLookahead = 3;
  for (int s = s0; s <= S && !stopped; ++s) {
    SCS_CHECK(epoch_launches(st, s, nullptr));
    if (s == S) break;
    SCS_HIP(hipEventRecord(tev[4 + s], st));
    epochs_launched = s + 1;
    if (s + 1 - s0 >= kLookahead) {
      const int q = s + 1 - kLookahead;
      SCS_HIP(hipEventSynchronize(tev[4 + q]));
      if (__atomic_load_n(ctx->stop_flags + q, __ATOMIC_ACQUIRE)) break;
    }
  }
  SCS_CHECK(launch_premap_batched(st, desc, nprob, 1, wout_dev));
  SCS_HIP(hipEventRecord(tev[3], st));
  std::vector<SolveState> hs(nprob);
  SCS_HIP(hipMemcpyAsync(hs.data(), states, sizeof(SolveState) * nprob, hipMemcpyDeviceToHost, st));
  SCS_HIP(hipStreamSynchronize(st));

  int worst = SCS_OK;
  float t_setup = 0.f, t_solve = 0.f;
  hipEventElapsedTime(&t_setup, tev[0], tev[1]);
  hipEventElapsedTime(&t_solve, tev[1], tev[3]);
  double t_inner = 0.0;  // shared inner-loop launches of every epoch enqueued (timing only)
  if (o.timing)
    for (int s = 0; s < epochs_launched; ++s) {
      float ms = 0.f;
      hipEventElapsedTime(&ms, tev[4 + S + s], tev[4 + s]);
      t_inner += ms;
    }
  for (int p = 0; p < nprob; ++p) {
    const SolveState& h = hs[sidx[p]];
    int status = SCS_OK;
    if (h.status == SCS_ENONFINITE || h.status == SCS_EDEVICE) status = h.status;
    else if (h.status == SCS_DIVERGED) status = SCS_DIVERGED;
    else if (o.stop_rule != SCS_STOP_EPOCHS && !h.done) status = SCS_NOT_CONVERGED;
    else if (rank_def[p]) status = SCS_SKETCH_RANK_DEFICIENT;
    if (status < 0) worst = std::min(worst, status);
    else if (worst >= 0) worst = std::max(worst, status);
    if (reports) {
      scs_report& r = reports[p];
      std::memset(&r, 0, sizeof(r));
      r.status = status;
      r.epochs = h.epochs;
      r.k_used = k_used[p];
      r.steps = m[p];
      r.eta = h.eta;
      r.beta_hat = h.beta_sum / (double)n[p];
      r.objective = h.obj;
      r.grad_norm = std::sqrt(h.gnorm2);
      r.certificate = h.cert;
      r.lam_top = h.lam_top;
      r.backoffs = h.backoffs;
      r.workgroups = W;
      r.ms_sketch = t_setup;
      r.ms_apply = 0.0;
      r.ms_solve = t_solve;
      r.ms_inner = t_inner;
      r.n_inner = o.timing ? epochs_launched : 0;
    }
  }
  if (worst == SCS_ENONFINITE) set_error("non-finite value in X or y of at least one problem");
  if (worst == SCS_EDEVICE) set_error("inner loop: a cross-workgroup wait exceeded its budget");
  return worst;
}

// The regularization path. reuse_sketch: the sketch buffers of the context already hold this X's
// sketch (an earlier stage of a warm-started path). W0 (device ny x d, nullable): start points in the
// original space, w~ = P_lambda^{1/2} w0 for every lambda of the call.
static int path_impl(scs_ctx* ctx, const float* X, int64_t n, int64_t d, int64_t ldx, const float* Y, int ny,
                     const double* lambdas, int nl, int k, double eps, const double* f_star, const scs_opts* opts,
                     float* W_out, scs_report* reports, bool reuse_sketch, const float* W0) {
  if (!ctx || !Y || !lambdas || !W_out || ny < 1 || nl < 1) {
    set_error("null argument, ny < 1 or nl < 1");
    return SCS_EINVAL;
  }
  SCS_CHECK(validate_problem(X, n, d, ldx, 1.0));
  scs_opts o;
  scs_opts_default(&o);
  if (opts) o = *opts;
  const int l = k + o.oversample;
  if (k < 0 || k > d || (k > 0 && (o.oversample < 0 || !sketch_width_ok(o, k, n, d))) || n + d > INT32_MAX) {
    set_error("need 0 <= k and, for k > 0, q (k + p) <= min(d, n, 136) for q Krylov blocks");
    return SCS_EINVAL;
  }
  for (int j = 0; j < nl; ++j)
    if (!(lambdas[j] > 0.0) || !std::isfinite(lambdas[j])) {
      set_error("every lambda must be a finite positive number");
      return SCS_EINVAL;
    }
  if (o.omega || o.indices || o.trace_w || (o.stop_rule == SCS_STOP_GAP && !f_star)) {
    set_error("path solve: omega, indices, trace_w must be NULL; the gap rule needs f_star for every solve");
    return SCS_EINVAL;
  }
  if (o.batch < 1 || o.batch > kInnerMaxB || o.max_epochs < 1 || o.steps < 0 || !(o.step_scale > 0.0) ||
      !(o.epoch_factor >= 0.0) || o.stop_rule < 0 || o.stop_rule > 2 || d > 16 * batched_max_slice(o.batch)) {
    set_error("bad options: need 1 <= batch <= 256, max_epochs >= 1, steps >= 0, step_scale > 0, and d <= 8192 "
              "(2048 for batch > 64, 1024 for batch > 128)");
    return SCS_EINVAL;
  }
  Guard g(ctx->device);
  free_retired(ctx);
  hipStream_t st = ctx->stream;
  const int P = nl * ny, b = o.batch, S = o.max_epochs, mixed = o.precision == SCS_PREC_MIXED;
  const int es = mixed ? 2 : 4;
  constexpr int G = 8;
  // W cooperating workgroups per solve: opts.workgroups when positive, else one per 256 columns
  // (measured on the 1024-column path: 256-column slices beat 512 and 128)
  const int64_t maxs = batched_max_slice(o.batch);
  const int W = (int)std::min<int64_t>(
      16, std::max<int64_t>(cdiv(d, maxs),
                            o.workgroups > 0 ? (int64_t)o.workgroups : cdiv(d, std::min<int64_t>(256, maxs))));
  const int64_t ldt = cdiv(d, mixed ? 128 : 64) * (mixed ? 128 : 64);
  const int64_t m = epoch_steps(o, n, b);
  const int64_t N = n + d;
  const int nblk = (int)std::max<int64_t>(1, std::min<int64_t>(1024, cdiv(n, 64)));  // residual row blocks
  if (o.implicit_apply && (mixed || d > 2048 || k > 128 || k < 1)) {
    set_error("implicit apply: needs FP32 precision, 1 <= k <= 128 and d <= 2048");
    return SCS_EINVAL;
  }

  // ---- workspace
  // materialized rows: one set per lambda; implicit: one padded copy of X shared by every lambda
  const int nsets = o.implicit_apply ? 1 : nl;
  void* xt_all = wsb(ctx, "p_xt", (size_t)nsets * n * ldt * es);
  void* reg_all = wsb(ctx, "p_reg", (size_t)nsets * d * ldt * es);
  if (!xt_all || !reg_all) return SCS_ENOMEM;
  WS(beta_all, float, "p_beta", (int64_t)nl * N);
  WS(cum_all, uint64_t, "p_cum", (int64_t)nl * N);
  WS(vec_all, float, "p_vec", (int64_t)4 * P * d);  // wt | wt_prev | w32 | mu, each P x d
  WS(tmp_all, double, "p_tmp", (int64_t)P * d);
  WS(gsum, double, "p_g", (int64_t)P * d);
  WS(rsq, double, "p_rsq", (int64_t)P * nblk);
  WS(R, float, "p_R", n * P);
  WS(idx_all, int32_t, "p_idx", (int64_t)P * G * m * b);
  WS(sc_all, float, "p_scale", (int64_t)P * G * m * b);
  WS(ut, float, "p_UT", std::max<int64_t>((int64_t)k * d, 1));
  WS(lam64, double, "p_lam", std::max(k, 1));
  WS(xbuf_all, uint64_t, "p_xbuf", (int64_t)P * inner_xbuf_words(W));
  WS(states, SolveState, "p_state", P);
  WS(done_count, int, "p_done", 1);
  WS(desc, BatchProb, "p_desc", P);
  WS(draw_pre, int64_t, "p_prefix", (int64_t)P + 1);
  WS(scr, double, "sampler_scratch", (size_t)sampler_scratch_len(N));
  constexpr int kPc = 128;  // problems per GEMM call (the MFMA kernels take up to 144 columns)
  // the residual matrix R (n x P, a workspace buffer) is the split-K GEMM's B operand, at column offsets
  // that are multiples of kPc: its rows are 16-byte aligned exactly when P is a multiple of 4
  const int64_t nch = gemm_tn_splitk_chunks(n, d, std::min(kPc, P), X, ldx, nullptr, P);
  const int64_t chunk = cdiv(n, nch), nchunks = cdiv(n, chunk);
  WS(part, float, "p_partial", nchunks * d * kPc);
  SCS_HIP(hipMemsetAsync(states, 0, sizeof(SolveState) * P, st));
  SCS_HIP(hipMemsetAsync(vec_all, 0, sizeof(float) * 2 * P * d, st));
  SCS_HIP(hipMemsetAsync(xbuf_all, 0, sizeof(uint64_t) * P * inner_xbuf_words(W), st));
  SCS_HIP(hipMemsetAsync(done_count, 0, sizeof(int), st));
  // tev: 0 start, 1-2 stage ends, 3 end, 4 + s end of epoch s (where the host reads stop flag s);
  // with timing, 4 + S + s opens the inner loop of epoch s
  SCS_CHECK(ensure_events(ctx, 0, (size_t)4 + (o.timing ? 2 * S : S)));
  SCS_CHECK(ensure_stop_flags(ctx, (size_t)S + 1));
  std::memset(ctx->stop_flags, 0, sizeof(int) * (S + 1));
  hipEvent_t* tev = ctx->tevents.data();
  SCS_HIP(hipEventRecord(tev[0], st));

  // ---- one sketch for every lambda (Alg. 2 does not involve lambda)
  int k_used = k;
  bool rank_def = false;
  if (k > 0 && !reuse_sketch) {
    SCS_CHECK(sketch_impl(ctx, X, n, d, ldx, k, o, true, &rank_def));
    if (rank_def) k_used = 0;
  }
  const bool implicit = o.implicit_apply && k_used > 0;
  if (k_used > 0) {
    SCS_HIP(hipMemcpyAsync(ut, ws<float>(ctx, "UT32", 0), sizeof(float) * k * d, hipMemcpyDeviceToDevice, st));
    SCS_HIP(hipMemcpyAsync(lam64, ws<double>(ctx, "lam", 0), sizeof(double) * k, hipMemcpyDeviceToDevice, st));
  }
  SCS_HIP(hipEventRecord(tev[1], st));
  // ---- per lambda: P_lambda^{-1/2} rows, smoothness and sampling tables (shared by its ny solves)
  float* xn2 = nullptr;
  if (implicit) {
    SCS_HIP(hipMemcpy2DAsync(xt_all, ldt * 4, X, ldx * 4, d * 4, n, hipMemcpyDeviceToDevice, st));
    xn2 = ws<float>(ctx, "p_xnorm2", n);
    if (!xn2) return SCS_ENOMEM;
    SCS_CHECK(launch_rownorm(st, X, n, d, ldx, xn2));
  }
  for (int j = 0; j < nl; ++j) {
    char* xt = (char*)xt_all + (size_t)(implicit ? 0 : j) * n * ldt * es;
    char* rg = (char*)reg_all + (size_t)(implicit ? 0 : j) * d * ldt * es;
    float* beta = beta_all + (int64_t)j * N;
    SolveState* st0 = states + (int64_t)j * ny;
    if (implicit) {
      SCS_CHECK(launch_implicit_beta(st, xn2, ws<float>(ctx, "Z", 0), gemm_wide_kpad(k_used), ut, lam64, k_used, n,
                                     d, lambdas[j], beta));
    } else if (k_used > 0) {
      SCS_CHECK(apply_impl(ctx, X, n, d, ldx, ws<float>(ctx, "U32", 0), ws<float>(ctx, "Z", 0), lam64, k_used,
                           lambdas[j], mixed, mixed, xt, rg, ldt, beta, st0));
    } else {
      if (mixed) {
        WS(tmp16, uint16_t, "xcopy16", n * d);
        SCS_CHECK(launch_copy_bf16(st, X, n, d, ldx, tmp16));
        SCS_HIP(hipMemcpy2DAsync(xt, ldt * 2, tmp16, d * 2, d * 2, n, hipMemcpyDeviceToDevice, st));
        SCS_CHECK(launch_rownorm_bf16(st, tmp16, n, d, beta));
      } else {
        SCS_HIP(hipMemcpy2DAsync(xt, ldt * 4, X, ldx * 4, d * 4, n, hipMemcpyDeviceToDevice, st));
        SCS_CHECK(launch_rownorm(st, X, n, d, ldx, beta));
      }
      WS(rtmp, float, "regtmp", d * d);
      SCS_CHECK(launch_fill_scaled_identity(st, d, std::sqrt((double)n * lambdas[j]), mixed, rtmp, beta + n));
      SCS_HIP(hipMemcpy2DAsync(rg, ldt * es, rtmp, d * es, d * es, d, hipMemcpyDeviceToDevice, st));
    }
    SCS_CHECK(launch_sampler_prepare(st, beta, N, cum_all + (int64_t)j * N, scr, sampler_scratch_len(N), st0,
                                     o.uniform_sampling));
    for (int r = 1; r < ny; ++r)
      SCS_HIP(hipMemcpyAsync(st0 + r, st0, sizeof(SolveState), hipMemcpyDeviceToDevice, st));
  }
  SCS_HIP(hipEventRecord(tev[2], st));

  // ---- descriptors: solve p = j ny + r
  std::vector<BatchProb> hp(P);
  std::vector<int64_t> dpre((size_t)P + 1, 0);
  const int64_t slice = cdiv(cdiv(d, W), 4) * 4;
  for (int p = 0; p < P; ++p) {
    const int j = p / ny, r = p % ny;
    BatchProb& q = hp[p];
    std::memset(&q, 0, sizeof(q));
    q.X = X;
    q.n = n;
    q.d = d;
    q.ldx = ldx;
    q.y = Y + (int64_t)r * n;
    q.lambda = lambdas[j];
    q.k = k_used;
    q.UT = k_used > 0 ? ut : nullptr;
    q.lam = k_used > 0 ? lam64 : nullptr;
    q.wt = vec_all + (int64_t)p * d;
    q.wt_prev = vec_all + (int64_t)(P + p) * d;
    q.w32 = vec_all + (int64_t)(2 * P + p) * d;
    q.mu = vec_all + (int64_t)(3 * P + p) * d;
    q.tmp = tmp_all + (int64_t)p * d;
    q.state = states + p;
    q.g64 = gsum + (int64_t)p * d;
    q.grows = 1;
    q.grsq = rsq + (int64_t)p * nblk;
    q.nwg = nblk;
    q.stop_rule = o.stop_rule;
    q.eps = eps;
    q.f_star = f_star ? f_star[p] : 0.0;
    q.cum = cum_all + (int64_t)j * N;
    q.N = N;
    q.draws = m * b;
    q.idx = idx_all + (int64_t)p * G * m * b;
    q.scale = sc_all + (int64_t)p * G * m * b;
    InnerArgs& a = q.inner;
    a.n = n;
    a.d = d;
    q.Z = implicit ? ws<float>(ctx, "Z", 0) : nullptr;
    q.ldz = gemm_wide_kpad(k_used);
    a.Xt = (char*)xt_all + (size_t)(implicit ? 0 : j) * n * ldt * es;
    a.ldx = ldt;
    a.reg = (char*)reg_all + (size_t)(implicit ? 0 : j) * d * ldt * es;
    a.ldr = ldt;
    a.mu = q.mu;
    a.m = m;
    a.b = b;
    a.eta_from_state = 1;
    a.step_scale = o.step_scale;
    a.average = o.average;
    a.W = W;
    a.xcd_stride = 1;
    a.slice = slice;
    a.wt = q.wt;
    a.wt_prev = q.wt_prev;
    a.xbuf = xbuf_all + (int64_t)p * inner_xbuf_words(W);
    a.state = q.state;
    dpre[p + 1] = dpre[p] + (int64_t)G * m * b;
  }
  SCS_HIP(hipMemcpyAsync(desc, hp.data(), sizeof(BatchProb) * P, hipMemcpyHostToDevice, st));
  SCS_HIP(hipMemcpyAsync(draw_pre, dpre.data(), sizeof(int64_t) * (P + 1), hipMemcpyHostToDevice, st));
  const float* W32 = vec_all + (int64_t)2 * P * d;
  if (W0) {
    for (int p = 0; p < P; ++p) {
      SCS_CHECK(launch_pmhalf_inv(st, k_used > 0 ? ut : nullptr, lam64, k_used, d, lambdas[p / ny], W0 + (int64_t)(p % ny) * d,
                                  hp[p].wt));
      SCS_HIP(hipMemcpyAsync(hp[p].wt_prev, hp[p].wt, sizeof(float) * d, hipMemcpyDeviceToDevice, st));
    }
  }

  // ---- epochs: the gradients of all P solves as two MFMA GEMMs over the shared X; once every solve
  // has stopped (epochs queued ahead of the host's stop decision, or the rest of a replayed graph)
  // they return at entry, as the per-solve kernels do
  Gate all_done;
  all_done.count = done_count;
  all_done.total = P;
  auto epoch_launches = [&](hipStream_t q, int s, const int* clk) -> int {
    SCS_CHECK(launch_premap_batched(q, desc, P, 0, nullptr));
    for (int c0 = 0; c0 < P; c0 += kPc) {
      const int pc = std::min(kPc, P - c0);
      SCS_CHECK(launch_gemm_nt_longk(q, 0, X, n, d, ldx, W32 + (int64_t)c0 * d, pc, d, R + c0, P, false, all_done));
    }
    SCS_CHECK(launch_residual_batched(q, R, n, P, Y, ny, nblk, rsq, all_done));
    for (int c0 = 0; c0 < P; c0 += kPc) {
      const int pc = std::min(kPc, P - c0);
      SCS_CHECK(launch_gemm_tn_splitk(q, 0, X, n, d, ldx, R + c0, pc, P, part, chunk, nchunks, all_done));
      SCS_CHECK(launch_reduce_partials_t(q, part, nchunks, d, pc, gsum + (int64_t)c0 * d, d, all_done));
    }
    SCS_CHECK(launch_grad_finalize_batched(q, desc, P, s == 0 ? 1 : 0, done_count,
                                           clk ? ctx->stop_flags : ctx->stop_flags + s, clk));
    if (!clk && s == S) return SCS_OK;
    const int slot = s % G;
    if (clk || slot == 0) SCS_CHECK(launch_sample_batched(q, desc, P, draw_pre, dpre[P], o.seed, s, G, clk));
    if (o.timing) SCS_HIP(hipEventRecord(tev[4 + S + s], q));
    if (implicit) SCS_CHECK(launch_inner_implicit_batched(q, desc, P, d, k_used, b, slot, s, clk));
    else SCS_CHECK(launch_inner_epoch_batched(q, desc, P, W, slice, b, mixed, slot, s, clk));
    if (clk) SCS_CHECK(launch_clock_advance(q, ctx_clock(ctx)));
    return SCS_OK;
  };
  int epochs_launched = 0;
  int s0 = 0;
  bool stopped = false;
  if (!o.no_graph && !o.timing) SCS_CHECK(run_epoch_graph(ctx, st, S, epoch_launches, &s0, &stopped));
  constexpr int kLookahead = 3;
  for (int s = s0; s <= S && !stopped; ++s) {
    SCS_CHECK(epoch_launches(st, s, nullptr));
    if (s == S) break;
    SCS_HIP(hipEventRecord(tev[4 + s], st));
    epochs_launched = s + 1;
    if (s + 1 - s0 >= kLookahead) {
      const int q = s + 1 - kLookahead;
      SCS_HIP(hipEventSynchronize(tev[4 + q]));
      if (__atomic_load_n(ctx->stop_flags + q, __ATOMIC_ACQUIRE)) break;
    }
  }
  std::vector<float*> wo(P);
  for (int p = 0; p < P; ++p) wo[p] = W_out + (int64_t)p * d;
  WS(wout_dev, float*, "p_wout", P);
  SCS_HIP(hipMemcpyAsync(wout_dev, wo.data(), sizeof(float*) * P, hipMemcpyHostToDevice, st));
  SCS_CHECK(launch_premap_batched(st, desc, P, 1, wout_dev));
  SCS_HIP(hipEventRecord(tev[3], st));
  std::vector<SolveState> hs(P);
  SCS_HIP(hipMemcpyAsync(hs.data(), states, sizeof(SolveState) * P, hipMemcpyDeviceToHost, st));
  SCS_HIP(hipStreamSynchronize(st));

  float t_sk = 0.f, t_ap = 0.f, t_so = 0.f;
  hipEventElapsedTime(&t_sk, tev[0], tev[1]);
  hipEventElapsedTime(&t_ap, tev[1], tev[2]);
  hipEventElapsedTime(&t_so, tev[2], tev[3]);
  double t_inner = 0.0;  // shared inner-loop launches of every epoch enqueued (timing only)
  if (o.timing)
    for (int s = 0; s < epochs_launched; ++s) {
      float ms = 0.f;
      hipEventElapsedTime(&ms, tev[4 + S + s], tev[4 + s]);
      t_inner += ms;
    }
  int worst = SCS_OK;
  for (int p = 0; p < P; ++p) {
    const SolveState& h = hs[p];
    int status = SCS_OK;
    if (h.status == SCS_ENONFINITE || h.status == SCS_EDEVICE) status = h.status;
    else if (h.status == SCS_DIVERGED) status = SCS_DIVERGED;
    else if (o.stop_rule != SCS_STOP_EPOCHS && !h.done) status = SCS_NOT_CONVERGED;
    else if (rank_def) status = SCS_SKETCH_RANK_DEFICIENT;
    if (status < 0) worst = std::min(worst, status);
    else if (worst >= 0) worst = std::max(worst, status);
    if (reports) {
      scs_report& rp = reports[p];
      std::memset(&rp, 0, sizeof(rp));
      rp.status = status;
      rp.epochs = h.epochs;
      rp.k_used = k_used;
      rp.steps = m;
      rp.eta = h.eta;
      rp.beta_hat = h.beta_sum / (double)n;
      rp.objective = h.obj;
      rp.grad_norm = std::sqrt(h.gnorm2);
      rp.certificate = h.cert;
      rp.lam_top = h.lam_top;
      rp.backoffs = h.backoffs;
      rp.workgroups = implicit ? 1 : W;
      rp.ms_sketch = t_sk;
      rp.ms_apply = t_ap;
      rp.ms_solve = t_so;
      rp.ms_inner = t_inner;
      rp.n_inner = o.timing ? epochs_launched : 0;
    }
  }
  if (worst == SCS_ENONFINITE) set_error("non-finite value in X or Y");
  if (worst == SCS_EDEVICE) set_error("inner loop: a cross-workgroup wait exceeded its budget");
  return worst;
}

int scs_svrg_solve_path(scs_ctx* ctx, const float* X, int64_t n, int64_t d, int64_t ldx, const float* Y, int ny,
                        const double* lambdas, int nl, int k, double eps, const double* f_star, const scs_opts* opts,
                        float* W_out, scs_report* reports) {
  scs_opts o;
  scs_opts_default(&o);
  if (opts) o = *opts;
  if (o.w0 || o.wt_out || o.epoch_offset != 0) {
    set_error("path solve: w0, wt_out and epoch_offset apply to single solves (use warm_start for the path)");
    return SCS_EINVAL;
  }
  if (!o.warm_start || nl == 1 || !W_out || ny < 1 || nl < 1 || !lambdas)
    return path_impl(ctx, X, n, d, ldx, Y, ny, lambdas, nl, k, eps, f_star, opts, W_out, reports, false, nullptr);
  // Continuation: lambda j's ny solves start from lambda j-1's solutions; one sketch for all lambdas.
  std::vector<scs_report> local(reports ? 0 : (size_t)ny);
  int worst = SCS_OK, k_stage = k;
  for (int j = 0; j < nl; ++j) {
    scs_report* rj = reports ? reports + (int64_t)j * ny : local.data();
    const int rc = path_impl(ctx, X, n, d, ldx, Y, ny, lambdas + j, 1, k_stage, eps, f_star ? f_star + (int64_t)j * ny : nullptr,
                             &o, W_out + (int64_t)j * ny * d, rj, j > 0 && k_stage > 0,
                             j > 0 ? W_out + (int64_t)(j - 1) * ny * d : nullptr);
    if (rc < 0) return rc;
    if (j == 0 && rj[0].k_used == 0) k_stage = 0;  // the sketch lost rank: the path continues with P = I
    if (worst >= 0) worst = std::max(worst, rc);
  }
  return worst;
}

}  // extern "C"
