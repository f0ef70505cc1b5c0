// Symmetric eigendecomposition of the l x l Rayleigh-Ritz matrix of the sketch (Alg. 2: the SVD of
// the projected block, here B = (XQ)^T (XQ) / n), in FP64, l = k + p <= 136:
//  1. Householder reduction to tridiagonal form, T = Qh^T B Qh, Qh = H_0 H_1 ... H_{l-3}
//     (one workgroup, B in LDS; reflector j is stored with its scale tau_j);
//  2. every eigenvalue of T by multisection on Sturm counts (G lanes per eigenvalue, so the
//     eigenvalues come out sorted);
//  3. the eigenvectors of T by inverse iteration with a partially pivoted LU of T - theta I (one
//     thread per eigenvector); members of groups of eigenvalues closer than 1e-10 ||T|| are redone
//     in sequence with the earlier members projected out at every iteration;
//  4. V = Qh Z by applying the reflectors to Z in reverse order (one workgroup, Z in LDS).
// The outputs follow the library's convention: theta[i] and column i of V (row-major l x l) form
// an eigenpair, order[r] is the index of the r-th largest eigenvalue.
#include "scs_internal.h"

namespace scs {

namespace {

constexpr int kEigThreads = 1024;
constexpr int kEigMaxL = 144;  // >= the largest sketch width

__device__ __forceinline__ double eig_block_sum(double v, double* sred) {
  v = wave_sum_d_fast(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sred[wave] = v;
  __syncthreads();
  double t = 0.0;
  for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += sred[q];
  return t;
}

// Reduction of B to tridiagonal form (lower variant): for j = 0 .. l-3 the reflector
// H_j = I - tau_j v v^T, v = (1, v_1, ..., v_{m-1}) acting on rows j+1 .. l-1, maps column j below
// the diagonal onto beta_j e_1; the trailing block is updated as A - v w^T - w v^T with
// w = tau A v - (tau^2 / 2)(v^T A v) v.
__device__ __forceinline__ void tridiag64_body(double* A /* LDS, l x l */, const double* B, int l, double* dd,
                                               double* ee, double* Vh, double* tau_out) {
  __shared__ double vv[kEigMaxL], ww[kEigMaxL];
  __shared__ double sred[kEigThreads / 64];
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, nwave = nt >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: loops over it stay scalar
  for (int e = tid; e < l * l; e += nt) A[e] = B[e];
  __syncthreads();
  // sigma of column j = sum of squares below its first sub-diagonal entry; for j + 1 it is gathered
  // during column j's rank-2 update (lane 0 of each wave updates column j + 1 of its rows) and the
  // partial sums travel with the update's closing barrier, so a column costs four barriers
  __shared__ double ssig[kEigThreads / 64];
  double sig;
  {
    double part = 0.0;
    for (int i = 2 + tid; i < l; i += nt) {
      const double x = A[i * l];
      part += x * x;
    }
    sig = eig_block_sum(part, sred);
  }
  for (int j = 0; j + 2 < l; ++j) {
    const int m = l - j - 1, r0 = j + 1;
    const double x0 = A[r0 * l + j];
    double beta = x0, tau = 0.0, scal = 0.0;
    if (sig > 0.0) {
      const double mu = sqrt(x0 * x0 + sig);
      beta = x0 <= 0.0 ? mu : -mu;
      tau = (beta - x0) / beta;
      scal = 1.0 / (x0 - beta);
    }
    for (int i = tid; i < m; i += nt) {
      const double v = i == 0 ? 1.0 : A[(r0 + i) * l + j] * scal;
      vv[i] = v;
      Vh[(int64_t)j * l + i] = v;
    }
    if (tid == 0) {
      dd[j] = A[j * l + j];
      ee[j] = beta;
      tau_out[j] = tau;
    }
    __syncthreads();
    if (tau == 0.0) {  // uniform: every thread holds the same tau; no update, sigma of j + 1 read directly
      double part = 0.0;
      for (int i = 2 + tid; i < m; i += nt) {
        const double x = A[(r0 + i) * l + r0];
        part += x * x;
      }
      sig = eig_block_sum(part, sred);
      continue;
    }
    // w = tau A v, with lane 0 of each wave adding up w_i v_i over its rows; each lane keeps its
    // entries of v (columns lane, lane + 64, lane + 128) in registers for the column
    constexpr int kVC = (kEigMaxL + 63) / 64;
    double vr[kVC];
#pragma unroll
    for (int q = 0; q < kVC; ++q) vr[q] = lane + 64 * q < m ? vv[lane + 64 * q] : 0.0;
    double pw = 0.0;
    for (int i = wave; i < m; i += nwave) {
      double acc = 0.0;
      const double* rowi = A + (r0 + i) * l + r0;
#pragma unroll
      for (int q = 0; q < kVC; ++q)
        if (lane + 64 * q < m) acc += rowi[lane + 64 * q] * vr[q];
      acc = wave_sum_d_fast(acc);
      if (lane == 0) {
        const double wi = tau * acc;
        ww[i] = wi;
        pw += wi * vv[i];
      }
    }
    if (lane == 0) sred[wave] = pw;
    __syncthreads();
    double pp = 0.0;
    for (int q = 0; q < nwave; ++q) pp += sred[q];
    const double al = -0.5 * tau * pp;
    for (int i = tid; i < m; i += nt) ww[i] += al * vv[i];
    __syncthreads();
    double ps = 0.0;
    double wr[kVC];
#pragma unroll
    for (int q = 0; q < kVC; ++q) wr[q] = lane + 64 * q < m ? ww[lane + 64 * q] : 0.0;
    for (int i = wave; i < m; i += nwave) {
      const double vi = vv[i], wi = ww[i];
      double* row = A + (r0 + i) * l + r0;
#pragma unroll
      for (int q = 0; q < kVC; ++q) {
        const int c = lane + 64 * q;
        if (c < m) {
          const double x = row[c] - (vi * wr[q] + wi * vr[q]);
          row[c] = x;
          if (c == 0 && i >= 2) ps += x * x;   // column j + 1 below its first sub-diagonal entry
        }
      }
    }
    if (lane == 0) ssig[wave] = ps;
    __syncthreads();
    sig = 0.0;
    for (int q = 0; q < nwave; ++q) sig += ssig[q];
  }
  if (tid == 0) {
    if (l >= 2) {
      dd[l - 2] = A[(l - 2) * l + l - 2];
      ee[l - 2] = A[(l - 1) * l + l - 2];
      tau_out[l - 2] = 0.0;
    }
    dd[l - 1] = A[(l - 1) * l + l - 1];
  }
}

// 1/q from the hardware estimate refined by two Newton steps (q is kept away from zero by pivmin).
__device__ __forceinline__ double recip_d(double q) {
  double r = __builtin_amdgcn_rcp(q);
  r = fma(r, fma(-q, r, 1.0), r);
  r = fma(r, fma(-q, r, 1.0), r);
  return r;
}

// Number of eigenvalues of T below x: negative pivots of the LDL^T factorization of T - x I.
__device__ __forceinline__ int sturm_count(const double* sd, const double* se2, int l, double x, double pivmin) {
  double q = sd[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  int cnt = q < 0.0;
#pragma unroll 8  // the broadcast LDS reads of several steps go out together
  for (int i = 1; i < l; ++i) {
    q = (sd[i] - x) - se2[i - 1] * recip_d(q);
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
}

// One inverse-iteration solve (T - th I) z_new = sc_in z on column t of zz (element i at [i * l + t]).
// The partially pivoted LU of T - th I is rebuilt inside the forward sweep (row interchange when the
// sub-diagonal entry is the larger; pivots below tiny in magnitude are raised to tiny, as inverse
// iteration wants), so that sweep reads only T and z; rows of U (reciprocal pivot, first and second
// super-diagonal) go to u0, u1, u2 at [i * l + t] for the backward sweep. Rows are processed in
// groups of kSolveRows whose loads are issued together (clamped indices keep them unconditional).
// Returns 1 / max|z_new|; *n2 receives sum z_new^2.
constexpr int kSolveRows = 8;

__device__ __forceinline__ double inv_solve(double* __restrict__ u0, double* __restrict__ u1,
                                            double* __restrict__ u2, const double* sd, const double* se,
                                            double th, double tiny, double* __restrict__ zz, int l, int t,
                                            double sc_in, double* n2) {
  double ca = sd[0] - th, cb = se[0];  // the carried row: entries at columns i and i + 1
  double cur = zz[t] * sc_in;
  for (int i0 = 0; i0 + 1 < l; i0 += kSolveRows) {
    double nxt[kSolveRows], na[kSolveRows], nb[kSolveRows], nc[kSolveRows];
#pragma unroll
    for (int j = 0; j < kSolveRows; ++j) {
      const int i = min(i0 + j, l - 2);
      nxt[j] = zz[(i + 1) * l + t];
      na[j] = sd[i + 1] - th;
      nb[j] = se[i + 1];  // zero for the last row
      nc[j] = se[i];
    }
#pragma unroll
    for (int j = 0; j < kSolveRows; ++j) {
      const int i = i0 + j;
      if (i + 1 >= l) break;  // uniform
      const bool s = fabs(ca) < fabs(nc[j]);
      double piv = s ? nc[j] : ca;
      if (fabs(piv) < tiny) piv = piv < 0.0 ? -tiny : tiny;
      const double r = recip_d(piv);
      const double m = (s ? ca : nc[j]) * r;
      const double v1 = s ? na[j] : cb;
      const double x = nxt[j] * sc_in;
      const double pa = s ? x : cur, pb = s ? cur : x;  // right-hand side of the pivot row, of the other
      const int o = i * l + t;
      u0[o] = r;
      u1[o] = v1;
      u2[o] = s ? nb[j] : 0.0;
      zz[o] = pa;
      cur = pb - m * pa;
      ca = (s ? cb : na[j]) - m * v1;
      cb = s ? -m * nb[j] : nb[j];
    }
  }
  {
    double piv = ca;
    if (fabs(piv) < tiny) piv = piv < 0.0 ? -tiny : tiny;
    const int o = (l - 1) * l + t;
    u0[o] = recip_d(piv);
    u1[o] = 0.0;
    u2[o] = 0.0;
    zz[o] = cur;
  }
  double z1 = 0.0, z2 = 0.0, nz = 0.0, ss = 0.0;
  for (int i0 = l - 1; i0 >= 0; i0 -= kSolveRows) {
    double a0[kSolveRows], a1[kSolveRows], a2[kSolveRows], zv[kSolveRows];
#pragma unroll
    for (int j = 0; j < kSolveRows; ++j) {
      const int o = max(i0 - j, 0) * l + t;
      a0[j] = u0[o];
      a1[j] = u1[o];
      a2[j] = u2[o];
      zv[j] = zz[o];
    }
#pragma unroll
    for (int j = 0; j < kSolveRows; ++j) {
      const int i = i0 - j;
      if (i < 0) break;  // uniform
      const double zi = (zv[j] - a1[j] * z1 - a2[j] * z2) * a0[j];
      zz[i * l + t] = zi;
      z2 = z1;
      z1 = zi;
      nz = fmax(nz, fabs(zi));
      ss += zi * zi;
    }
  }
  *n2 = ss;
  return nz > 0.0 ? 1.0 / nz : 1.0;
}

__device__ void start_vector(double* zz, int l, int t) {
  for (int i = 0; i < l; ++i)
    zz[(int64_t)i * l + t] = 1.0 + 0.25 * (double)(((uint32_t)(i + 1) * 2654435761u + (uint32_t)t * 40503u) % 997u) / 997.0;
}

__device__ void scale_col(double* zz, int l, int t, double sc) {
  for (int i = 0; i < l; ++i) zz[(int64_t)i * l + t] *= sc;
}

__device__ void normalize2(double* zz, int l, int t) {
  double n2 = 0.0;
  for (int i = 0; i < l; ++i) n2 += zz[(int64_t)i * l + t] * zz[(int64_t)i * l + t];
  scale_col(zz, l, t, n2 > 0.0 ? 1.0 / sqrt(n2) : 0.0);
}

// Eigenpairs of the symmetric tridiagonal T (diagonal dd, off-diagonal ee). The vectors live in
// LDS; the rows of U of the solves (3 l^2 doubles) follow them in LDS when ULDS, else they go to work.
template <bool ULDS>
__device__ __forceinline__ void tridiag_eig_body(double* zz /* LDS: l x l vectors (element i of vector t at
                                                 [i * l + t]), then 3 l^2 rows of U when ULDS */,
                                                 const double* dd, const double* ee, int l, double* theta,
                                                 double* Z, double* work) {
  __shared__ double sd[kEigMaxL], se[kEigMaxL], se2[kEigMaxL], sth[kEigMaxL], csc[kEigMaxL];
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = tid; i < l; i += nt) {
    sd[i] = dd[i];
    const double e = i + 1 < l ? ee[i] : 0.0;
    se[i] = e;
    se2[i] = e * e;
  }
  __syncthreads();
  // Gershgorin interval and the scale of T (every thread, identical results)
  double lo = 0.0, hi = 0.0, nrm = 0.0, maxe2 = 0.0;
  for (int i = 0; i < l; ++i) {
    const double r = (i > 0 ? fabs(se[i - 1]) : 0.0) + (i + 1 < l ? fabs(se[i]) : 0.0);
    lo = i == 0 ? sd[i] - r : fmin(lo, sd[i] - r);
    hi = i == 0 ? sd[i] + r : fmax(hi, sd[i] + r);
    nrm = fmax(nrm, fabs(sd[i]) + r);
    if (i + 1 < l) maxe2 = fmax(maxe2, se2[i]);
  }
  if (nrm == 0.0) nrm = 1.0;
  const double pivmin = 1e-290 * fmax(1.0, maxe2);
  const double abstol = 1e-16 * nrm;
  // rows of U of each thread's solve, element i of thread t at [i * l + t] (coalesced across threads)
  const int64_t L2 = (int64_t)l * l;
  double* ub = ULDS ? zz + L2 : work;
  double* u0 = ub;
  double* u1 = ub + L2;
  double* u2 = ub + 2 * L2;
  // The t-th smallest eigenvalue by multisection: G lanes of one wave (G a power of two) evaluate
  // the Sturm count at G interior points of [a, b] together and keep the subinterval where the
  // count passes t, so count(a) <= t < count(b) holds throughout and [a, b] shrinks (G+1)-fold
  // per round.
  const int G = l <= 128 ? 8 : (l <= 256 ? 4 : 1);  // more lanes only add FP64 issue pressure on the CU
  const int lane = tid & 63;
  if (tid < G * l) {
    const int t = tid / G, s = tid % G;
    double a = lo - abstol, b = hi + abstol;
    for (int it = 0; it < 200; ++it) {
      const double h = (b - a) / (double)(G + 1);
      if (b - a <= fmax(abstol, 4.4e-16 * fmax(fabs(a), fabs(b))) || h <= 0.0 || a + h <= a) break;
      const double x = a + (double)(s + 1) * h;
      const bool above = sturm_count(sd, se2, l, x, pivmin) > t;
      // lanes of this eigenvalue: [base, base + G) of the wave
      const int base = lane - s;
      const uint64_t mask = (uint64_t)__ballot(above) >> base;
      const uint64_t mine = G == 64 ? mask : (mask & ((1ull << G) - 1ull));
      const int first = mine ? __builtin_ctzll(mine) : G;  // first point with count > t
      const double na = first == 0 ? a : a + (double)first * h;
      const double nb = first == G ? b : a + (double)(first + 1) * h;
      a = na;
      b = nb;
    }
    if (s == 0) {
      sth[t] = 0.5 * (a + b);
      theta[t] = 0.5 * (a + b);
    }
  }
  __syncthreads();
  // a zero pivot (th is an eigenvalue) is replaced by a tiny multiple of ||T||
  const double tiny = 1e-15 * nrm;
  if (tid < l) {
    // three solves from a fixed start vector (different per thread); the max-norm scaling of each
    // result is applied as the next solve reads it, the final 2-norm scaling on the way out
    const int t = tid;
    const double th = sth[t];
    start_vector(zz, l, t);
    double sc = 1.0, n2 = 0.0;
    for (int rep = 0; rep < 3; ++rep) sc = inv_solve(u0, u1, u2, sd, se, th, tiny, zz, l, t, sc, &n2);
    csc[t] = n2 > 0.0 ? 1.0 / sqrt(n2) : 0.0;
  }
  __syncthreads();
  // Eigenvalues within 1e-10 ||T|| of their predecessor do not determine their inverse-iteration
  // vectors individually: those are recomputed one after another (thread 0), projecting out the
  // earlier members of the group at every iteration, so the group's vectors come out orthonormal.
  const double ortol = 1e-10 * nrm;
  for (int t = 1; t < l; ++t) {
    if (sth[t] - sth[t - 1] > ortol) continue;  // uniform
    if (tid == 0) {
      int g0 = t - 1;
      while (g0 > 0 && sth[g0] - sth[g0 - 1] <= ortol) --g0;
      for (int j = g0; j < t; ++j) {  // earlier members in unit 2-norm, in place
        if (csc[j] != 1.0) scale_col(zz, l, j, csc[j]);
        csc[j] = 1.0;
      }
      start_vector(zz, l, t);
      for (int rep = 0; rep < 3; ++rep) {
        double n2 = 0.0;
        scale_col(zz, l, t, inv_solve(u0, u1, u2, sd, se, sth[t], tiny, zz, l, t, 1.0, &n2));
        for (int j = g0; j < t; ++j) {
          double dot = 0.0;
          for (int i = 0; i < l; ++i) dot += zz[(int64_t)i * l + j] * zz[(int64_t)i * l + t];
          for (int i = 0; i < l; ++i) zz[(int64_t)i * l + t] -= dot * zz[(int64_t)i * l + j];
        }
        normalize2(zz, l, t);
      }
      csc[t] = 1.0;
    }
    __syncthreads();
  }
  for (int e = tid; e < l * l; e += nt) {
    const int i = e / l;
    Z[e] = zz[e] * csc[e - i * l];
  }
}

// V = Qh Z = H_0 (H_1 (... (H_{l-3} Z))): reflector j acts on rows j+1 .. l-1. Z in LDS; each
// column dot is split over `parts` threads.
__device__ __forceinline__ void backtransform64_body(double* Zs /* LDS, l x l */, const double* Zin,
                                                     const double* Vh, const double* tau, int l, double* V,
                                                     const double* theta, int* order) {
  __shared__ double vv[kEigMaxL], wcol[kEigMaxL];
  __shared__ double red[8][kEigMaxL];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int parts = nt / l < 8 ? nt / l : 8;
  for (int e = tid; e < l * l; e += nt) Zs[e] = Zin[e];
  __syncthreads();
  for (int j = l - 3; j >= 0; --j) {
    const double tj = tau[j];
    if (tj == 0.0) continue;  // uniform
    const int m = l - j - 1, r0 = j + 1;
    for (int i = tid; i < m; i += nt) vv[i] = Vh[(int64_t)j * l + i];
    __syncthreads();
    if (tid < parts * l) {
      const int c = tid % l, pt = tid / l;
      double acc = 0.0;
      for (int i = pt; i < m; i += parts) acc += vv[i] * Zs[(r0 + i) * l + c];
      red[pt][c] = acc;
    }
    __syncthreads();
    for (int c = tid; c < l; c += nt) {
      double s = 0.0;
      for (int pt = 0; pt < parts; ++pt) s += red[pt][c];
      wcol[c] = tj * s;
    }
    __syncthreads();
    const int lane = tid & 63, nwave = nt >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    constexpr int kWC = (kEigMaxL + 63) / 64;  // each lane's entries of w (columns lane + 64 q) in registers
    double wr[kWC];
#pragma unroll
    for (int q = 0; q < kWC; ++q) wr[q] = lane + 64 * q < l ? wcol[lane + 64 * q] : 0.0;
    for (int i = wave; i < m; i += nwave) {
      const double vi = vv[i];
      double* row = Zs + (r0 + i) * l;
#pragma unroll
      for (int q = 0; q < kWC; ++q)
        if (lane + 64 * q < l) row[lane + 64 * q] -= vi * wr[q];
    }
    __syncthreads();
  }
  for (int e = tid; e < l * l; e += nt) V[e] = Zs[e];
  // theta ascending: the r-th largest is index l - 1 - r
  for (int r = tid; r < l; r += nt) order[r] = l - 1 - r;
  (void)theta;
}

// One-problem kernels and their batched forms (one workgroup per problem, its arguments from jobs).
__global__ __launch_bounds__(kEigThreads) void tridiag64_kernel(const double* B, int l, double* dd, double* ee,
                                                                double* Vh, double* tau_out) {
  extern __shared__ double dyn[];
  tridiag64_body(dyn, B, l, dd, ee, Vh, tau_out);
}

template <bool ULDS>
__global__ __launch_bounds__(kEigThreads) void tridiag_eig_kernel(const double* dd, const double* ee, int l,
                                                                  double* theta, double* Z, double* work) {
  extern __shared__ double dyn[];
  tridiag_eig_body<ULDS>(dyn, dd, ee, l, theta, Z, work);
}

__global__ __launch_bounds__(kEigThreads) void backtransform64_kernel(const double* Zin, const double* Vh,
                                                                      const double* tau, int l, double* V,
                                                                      const double* theta, int* order) {
  extern __shared__ double dyn[];
  backtransform64_body(dyn, Zin, Vh, tau, l, V, theta, order);
}

// the layout of a problem's work array (eig64_work_len(l) doubles), as launch_eig64 uses it
struct EigWork {
  double *Vh, *dd, *ee, *tau, *Zt, *tw;
  __host__ __device__ EigWork(double* work, int l) {
    Vh = work;
    dd = work + (int64_t)l * l;
    ee = dd + l;
    tau = ee + l;
    Zt = tau + l;
    tw = Zt + (int64_t)l * l;
  }
};

__global__ __launch_bounds__(kEigThreads) void tridiag64_batched_kernel(const Eig64Job* jobs) {
  extern __shared__ double dyn[];
  const Eig64Job j = jobs[blockIdx.x];
  const EigWork w(j.work, j.l);
  tridiag64_body(dyn, j.B, j.l, w.dd, w.ee, w.Vh, w.tau);
}

template <bool ULDS>
__global__ __launch_bounds__(kEigThreads) void tridiag_eig_batched_kernel(const Eig64Job* jobs) {
  extern __shared__ double dyn[];
  const Eig64Job j = jobs[blockIdx.x];
  const EigWork w(j.work, j.l);
  tridiag_eig_body<ULDS>(dyn, w.dd, w.ee, j.l, j.theta, w.Zt, w.tw);
}

__global__ __launch_bounds__(kEigThreads) void backtransform64_batched_kernel(const Eig64Job* jobs) {
  extern __shared__ double dyn[];
  const Eig64Job j = jobs[blockIdx.x];
  const EigWork w(j.work, j.l);
  backtransform64_body(dyn, w.Zt, w.Vh, w.tau, j.l, j.V, j.theta, j.order);
}

int g_max_lds_eig = -1;

int max_lds_eig() {
  if (g_max_lds_eig < 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return 65536;
    g_max_lds_eig = (int)prop.sharedMemPerBlock;
  }
  return g_max_lds_eig;
}

}  // namespace

int eig64_work_len(int l) { return 5 * l * l + 4 * l; }

int launch_eig64(hipStream_t st, const double* B, int l, double* work, double* V, double* theta, int* order) {
  const size_t bytes = (size_t)l * l * sizeof(double);
  if (l < 1 || l > kEigMaxL || (int64_t)bytes + 16384 > max_lds_eig()) {
    set_error("eigendecomposition: the sketch width k + p must be in [1, 136]");
    return SCS_EINVAL;
  }
  // l x l reflectors, the diagonal, off-diagonal and reflector scales (l each), the l x l vectors of T,
  // then 3 l^2 for the rows of U of the inverse-iteration solves
  const EigWork w(work, l);
  double *Vh = w.Vh, *dd = w.dd, *ee = w.ee, *tau = w.tau, *Zt = w.Zt, *tw = w.tw;
  if (bytes > 65536) {
    SCS_HIP(hipFuncSetAttribute((const void*)tridiag64_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    SCS_HIP(hipFuncSetAttribute((const void*)backtransform64_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)bytes));
  }
  tridiag64_kernel<<<1, 512, bytes, st>>>(B, l, dd, ee, Vh, tau);  // 512 threads: fewer waves at each barrier
  SCS_HIP(hipGetLastError());
  // the rows of U of the inverse-iteration solves join the vectors in LDS when both fit
  const size_t ebytes = 4 * bytes;
  if ((int64_t)ebytes + 8192 <= max_lds_eig()) {  // static LDS: 5760 bytes
    if (ebytes > 65536)
      SCS_HIP(hipFuncSetAttribute((const void*)tridiag_eig_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)ebytes));
    tridiag_eig_kernel<true><<<1, kEigThreads, ebytes, st>>>(dd, ee, l, theta, Zt, tw);
  } else {
    if (bytes > 65536)
      SCS_HIP(hipFuncSetAttribute((const void*)tridiag_eig_kernel<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)bytes));
    tridiag_eig_kernel<false><<<1, kEigThreads, bytes, st>>>(dd, ee, l, theta, Zt, tw);
  }
  SCS_HIP(hipGetLastError());
  backtransform64_kernel<<<1, kEigThreads, bytes, st>>>(Zt, Vh, tau, l, V, theta, order);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

int launch_eig64_batched(hipStream_t st, const Eig64Job* jobs, int njobs, int max_l) {
  if (njobs <= 0) return SCS_OK;
  const size_t bytes = (size_t)max_l * max_l * sizeof(double);
  if (max_l < 1 || max_l > kEigMaxL || (int64_t)bytes + 16384 > max_lds_eig()) {
    set_error("eigendecomposition: the sketch width k + p must be in [1, 136]");
    return SCS_EINVAL;
  }
  if (bytes > 65536) {
    SCS_HIP(hipFuncSetAttribute((const void*)tridiag64_batched_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)bytes));
    SCS_HIP(hipFuncSetAttribute((const void*)backtransform64_batched_kernel,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  }
  tridiag64_batched_kernel<<<(unsigned)njobs, 512, bytes, st>>>(jobs);
  SCS_HIP(hipGetLastError());
  const size_t ebytes = 4 * bytes;
  if ((int64_t)ebytes + 8192 <= max_lds_eig()) {
    if (ebytes > 65536)
      SCS_HIP(hipFuncSetAttribute((const void*)tridiag_eig_batched_kernel<true>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)ebytes));
    tridiag_eig_batched_kernel<true><<<(unsigned)njobs, kEigThreads, ebytes, st>>>(jobs);
  } else {
    if (bytes > 65536)
      SCS_HIP(hipFuncSetAttribute((const void*)tridiag_eig_batched_kernel<false>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    tridiag_eig_batched_kernel<false><<<(unsigned)njobs, kEigThreads, bytes, st>>>(jobs);
  }
  SCS_HIP(hipGetLastError());
  backtransform64_batched_kernel<<<(unsigned)njobs, kEigThreads, bytes, st>>>(jobs);
  SCS_HIP(hipGetLastError());
  return SCS_OK;
}

}  // namespace scs
