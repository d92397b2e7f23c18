// Lanczos iteration kernels, batched over the problems of one call.
//
// All per-problem control lives on the device (LzCtrl): the current Krylov
// index j, the stop flag, the Ritz value history.  The host only launches a
// fixed sequence of kernels per iteration and reads the stop flags once per
// chunk of iterations, so the sequence is the same for every iteration.
//
// Reductions are two-stage and deterministic: kLzBlocks partial sums per
// problem in fixed positions, then one workgroup adds them in a fixed tree.
//
// Iteration j (current vector v = q_j, w = H q_j on entry):
//   w -= sigma q_j (j > 0; sigma = alpha_0), |w|^2 before projection
//   c = Q^T w over q_0..q_j, alpha_j = c_j + sigma, w -= Q c, |w|^2 after
//       (classical Gram-Schmidt; it contains the three-term step, since the
//       coefficients of q_j and q_{j-1} are alpha_j - sigma and beta_{j-1})
//   only if |w| after < eta |w| before (or j = 0):
//       c = Q^T w, w -= Q c, |w|^2                      (second pass)
//   beta_j = |w|; lowest Ritz pair (theta, y) of T_{j+1}; stop test;
//   otherwise q_{j+1} = w / beta_j.
// One pass leaves w orthogonal to Q up to about eps |w before| / |w after|
// (relative), so the second pass is needed only when the projection removes
// most of w (the criterion of Daniel, Gragg, Kaufman and Stewart, here with
// eta = 0.1, i.e. at most ~10 eps per step).  The shift matters: the effective
// Hamiltonian carries the environments' energy as a large constant, and
// without it |H q_j| would exceed beta_j by orders of magnitude every step.  It
// is applied to w as its own rounding step before the projection, so that the
// rounding error of the subtraction is projected out as well.
//
// The basis rows, v and w have the padded length ld (a multiple of
// kLzAlign elements, zero beyond N), so every block's element range starts on
// a 16-byte boundary and the streaming kernels use 16-byte loads.  The
// dot-product kernel keeps its block's slice of w in LDS and streams the
// basis rows past it, so the basis is read once per pass and w once.
//
// With an FP32 basis (LzProblem::Qf set: the first pass of a mixed solve), rows
// 1.. are stored rounded to FP32 and v is set to exactly the stored row, so
// the Lanczos relation holds for the stored vectors up to beta_j times the
// rounding of q_{j+1}; row 0, the pass's start vector, stays FP64, so the Ritz
// vector's FP32 part is only the correction the pass adds.  All arithmetic
// stays FP64.
#include "internal.h"

namespace idmrg {
namespace {

constexpr int TB = 256;

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Deterministic block sum of one value per thread (TB threads): fixed tree.
__device__ double block_sum(double x, double* sh) {
  sh[threadIdx.x] = x;
  __syncthreads();
  for (int s = TB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ void range_of(int64_t N, int b, int64_t& lo, int64_t& hi) {
  const int64_t per = (N + kLzBlocks - 1) / kLzBlocks;
  lo = per * b;
  hi = lo + per;
  if (hi > N) hi = N;
  if (lo > N) lo = N;
}

// which: 0 = v, 1 = w, 2 = psi, 3 = s0
__device__ __forceinline__ double* vec_of(const LzProblem& p, int which) {
  return which == 0 ? p.v : (which == 1 ? p.w : (which == 2 ? p.psi : p.s0));
}

// partial[p][0][b] = sum_{n in range b} x[n] * y[n]
__global__ __launch_bounds__(TB) void k_dot_partial(const LzProblem* probs, const int32_t* active, int wx, int wy,
                                                    double* partial, int kmax) {
  __shared__ double sh[TB];
  const int p = blockIdx.y, b = blockIdx.x;
  if (active && !active[p]) return;
  const LzProblem pr = probs[p];
  const double* x = vec_of(pr, wx);
  const double* y = vec_of(pr, wy);
  int64_t lo, hi;
  range_of(pr.N, b, lo, hi);
  double acc = 0.0;
  for (int64_t n = lo + threadIdx.x; n < hi; n += TB) acc += x[n] * y[n];
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[((int64_t)p * kmax) * kLzBlocks + b] = acc;
}

// Sum kLzBlocks partials of slot i of each problem in a fixed tree.
__device__ double sum_partials(const double* partial, int p, int i, int kmax, double* sh) {
  double x = 0.0;
  for (int b = threadIdx.x; b < kLzBlocks; b += TB) x += partial[((int64_t)p * kmax + i) * kLzBlocks + b];
  return block_sum(x, sh);
}

constexpr double kReorthEta2 = 0.01;   // eta^2 of the second-pass criterion

// mode 1: beta_j = sqrt(sum) (after a second pass, where there was one);
// mode 2: norm0 = sqrt(sum);  mode 3: residual = sqrt(sum);  mode 5: overlap0 = |sum|;
// mode 4 (after the first pass): beta_j = sqrt(sum), and ctrl.reorth =
// cgs2 or j == 0 or sum < eta^2 |w before|^2 (pnorm).
__global__ __launch_bounds__(TB) void k_finalize(LzCtrl* ctrl, const int32_t* active, const double* partial,
                                                 const double* pnorm, int kmax, int mode, int cgs2 = 0) {
  __shared__ double sh[TB];
  const int p = blockIdx.x;
  if (active && !active[p]) return;
  if (mode == 1 && !ctrl[p].reorth) return;
  const double s = sum_partials(partial, p, 0, kmax, sh);
  double before = 0.0;
  if (mode == 4) {
    double x = 0.0;
    for (int b = threadIdx.x; b < kLzBlocks; b += TB) x += pnorm[(int64_t)p * kLzBlocks + b];
    before = block_sum(x, sh);
  }
  if (threadIdx.x == 0) {
    LzCtrl& c = ctrl[p];
    if (mode == 1 || mode == 4) c.beta_j = sqrt(s);
    if (mode == 4) {
      c.reorth = cgs2 || c.j == 0 || s < kReorthEta2 * before;
      c.reorths += c.reorth;
    }
    if (mode == 2) c.norm0 = sqrt(s);
    if (mode == 3) c.residual = sqrt(s);
    if (mode == 5) c.overlap0 = fabs(s);
  }
}

// v = Q[0] = psi / norm0 and zero padding of v, Q[0], w beyond N
// (problems with kcap == 0 sit this run out)
__global__ __launch_bounds__(TB) void k_start(const LzProblem* probs, const LzCtrl* ctrl) {
  const int p = blockIdx.y;
  if (ctrl[p].kcap == 0) return;
  const LzProblem pr = probs[p];
  const double inv = 1.0 / ctrl[p].norm0;
  for (int64_t n = blockIdx.x * (int64_t)TB + threadIdx.x; n < pr.ld; n += (int64_t)gridDim.x * TB) {
    const double x = n < pr.N ? pr.psi[n] * inv : 0.0;
    pr.v[n] = x;
    pr.Q[n] = x;
    if (n >= pr.N) pr.w[n] = 0.0;
  }
}

typedef double v2d __attribute__((ext_vector_type(2)));

// Element range [lo, hi) of block b over a padded vector of length ld.
__device__ __forceinline__ void pad_range(int64_t ld, int b, int64_t& lo, int64_t& hi) {
  int64_t per = (ld + kLzBlocks - 1) / kLzBlocks;
  per = (per + kLzAlign - 1) / kLzAlign * kLzAlign;
  lo = per * b;
  if (lo > ld) lo = ld;
  hi = lo + per;
  if (hi > ld) hi = ld;
}

constexpr int kSub = 4096;   // elements of w staged in LDS at a time

// partial[p][i][b] = sum_{n in range b} Q[i][n] w[n], i = 0..j.
// The block's slice of w goes through LDS kSub elements at a time; wave k
// takes rows i = k, k + 4, ... and adds its row sums into acc[i] in a fixed
// order, so the result does not depend on scheduling.
// Pass 0 first replaces w by w - sigma v (j > 0) while staging it, and puts
// the block's |w|^2 into pnorm[p][b]; pass 1 runs only where ctrl.reorth is set.
__global__ __launch_bounds__(TB) void k_mdot(const LzProblem* probs, const LzCtrl* ctrl, const int32_t* active,
                                             double* partial, double* pnorm, int kmax, int pass) {
  __shared__ __attribute__((aligned(16))) double xs[kSub];
  __shared__ double acc[kLzMaxK];
  __shared__ double sh[TB];
  const int p = blockIdx.y, b = blockIdx.x;
  if (!active[p] || (pass == 1 && !ctrl[p].reorth)) return;
  const LzProblem pr = probs[p];
  const int j = ctrl[p].j;
  const double sigma = pass == 0 && j > 0 ? ctrl[p].shift : 0.0;
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  int64_t lo, hi;
  pad_range(pr.ld, b, lo, hi);
  for (int i = t; i <= j; i += TB) acc[i] = 0.0;
  double nb = 0.0;
  for (int64_t s0 = lo; s0 < hi; s0 += kSub) {
    const int len = (int)(hi - s0 < kSub ? hi - s0 : kSub);
    __syncthreads();   // previous slice fully consumed (and acc initialised)
    for (int e = 2 * t; e < len; e += 2 * TB) {
      v2d x = *reinterpret_cast<const v2d*>(&pr.w[s0 + e]);
      if (sigma != 0.0) {
        const v2d vv = *reinterpret_cast<const v2d*>(&pr.v[s0 + e]);
        x.x -= sigma * vv.x;
        x.y -= sigma * vv.y;
        *reinterpret_cast<v2d*>(&pr.w[s0 + e]) = x;
      }
      nb += x.x * x.x + x.y * x.y;
      *reinterpret_cast<v2d*>(&xs[e]) = x;
    }
    __syncthreads();
    for (int i = wave; i <= j; i += TB / 64) {
      double a = 0.0;
      if (i == 0 || !pr.Qf) {
        const double* q = pr.Q + (int64_t)i * pr.ld + s0;
#pragma unroll 4
        for (int e = 2 * lane; e < len; e += 128) {
          const v2d qv = *reinterpret_cast<const v2d*>(&q[e]);
          const v2d xv = *reinterpret_cast<const v2d*>(&xs[e]);
          a += qv.x * xv.x + qv.y * xv.y;
        }
      } else {
        // FP32 row: four elements per 16-byte load (len is a multiple of kLzAlign)
        const float* q = pr.Qf + (int64_t)(i - 1) * pr.ld + s0;
#pragma unroll 2
        for (int e = 4 * lane; e < len; e += 256) {
          const float4 qv = *reinterpret_cast<const float4*>(&q[e]);
          const v2d x0 = *reinterpret_cast<const v2d*>(&xs[e]);
          const v2d x1 = *reinterpret_cast<const v2d*>(&xs[e + 2]);
          a += (double)qv.x * x0.x + (double)qv.y * x0.y + (double)qv.z * x1.x + (double)qv.w * x1.y;
        }
      }
      a = wave_sum(a);
      if (lane == 0) acc[i] += a;
    }
  }
  __syncthreads();
  for (int i = t; i <= j; i += TB) partial[((int64_t)p * kmax + i) * kLzBlocks + b] = acc[i];
  if (pass == 0) {
    nb = block_sum(nb, sh);
    if (t == 0) pnorm[(int64_t)p * kLzBlocks + b] = nb;
  }
}

// coef[p][i] = sum_b partial[p][i][b], i = 0..j; one block per (i, p).
// Pass 0: alpha_j = coef_j + sigma (and sigma = alpha_0 from j = 0);
// pass 1 runs only where ctrl.reorth is set.
__global__ __launch_bounds__(TB) void k_mdot_finalize(LzCtrl* ctrl, const int32_t* active, const double* partial,
                                                      double* coef, double* alpha, int kmax, int pass) {
  __shared__ double sh[TB];
  const int p = blockIdx.y, i = blockIdx.x;
  if (!active[p] || i > ctrl[p].j || (pass == 1 && !ctrl[p].reorth)) return;
  const double s = sum_partials(partial, p, i, kmax, sh);
  if (threadIdx.x == 0) {
    coef[(int64_t)p * kmax + i] = s;
    if (pass == 0 && i == ctrl[p].j) {
      const int j = ctrl[p].j;
      alpha[(int64_t)p * kmax + i] = s + (j > 0 ? ctrl[p].shift : 0.0);
      if (j == 0) ctrl[p].shift = s;
    }
  }
}

// w -= sum_{i<=j} coef_i Q[i] over the padded length, and
// partial[p][0][b] = |w|^2 over the block's range (after the update).
// Pass 1 runs only where ctrl.reorth is set.
__global__ __launch_bounds__(TB) void k_update(const LzProblem* probs, const LzCtrl* ctrl, const int32_t* active,
                                               const double* coef, double* partial, int kmax, int pass) {
  __shared__ double cs[kLzMaxK];
  __shared__ double sh[TB];
  const int p = blockIdx.y, b = blockIdx.x;
  if (!active[p] || (pass == 1 && !ctrl[p].reorth)) return;
  const LzProblem pr = probs[p];
  const int j = ctrl[p].j;
  const int t = threadIdx.x;
  for (int i = t; i <= j; i += TB) cs[i] = coef[(int64_t)p * kmax + i];
  __syncthreads();
  int64_t lo, hi;
  pad_range(pr.ld, b, lo, hi);
  double nrm = 0.0;
  if (!pr.Qf) {
    for (int64_t n = lo + 2 * t; n < hi; n += 2 * TB) {
      v2d s = {0.0, 0.0};
      const double* q = pr.Q + n;
#pragma unroll 4
      for (int i = 0; i <= j; ++i) {
        const v2d qv = *reinterpret_cast<const v2d*>(&q[(int64_t)i * pr.ld]);
        s.x += cs[i] * qv.x;
        s.y += cs[i] * qv.y;
      }
      v2d wv = *reinterpret_cast<const v2d*>(&pr.w[n]);
      wv.x -= s.x;
      wv.y -= s.y;
      *reinterpret_cast<v2d*>(&pr.w[n]) = wv;
      nrm += wv.x * wv.x + wv.y * wv.y;
    }
  } else {
    // FP64 row 0, FP32 rows 1..j; four elements per thread (hi - lo is a multiple of kLzAlign)
    for (int64_t n = lo + 4 * t; n < hi; n += 4 * TB) {
      const v2d q0a = *reinterpret_cast<const v2d*>(&pr.Q[n]);
      const v2d q0b = *reinterpret_cast<const v2d*>(&pr.Q[n + 2]);
      double s0 = cs[0] * q0a.x, s1 = cs[0] * q0a.y, s2 = cs[0] * q0b.x, s3 = cs[0] * q0b.y;
      const float* q = pr.Qf + n;
#pragma unroll 4
      for (int i = 1; i <= j; ++i) {
        const float4 qv = *reinterpret_cast<const float4*>(&q[(int64_t)(i - 1) * pr.ld]);
        s0 += cs[i] * (double)qv.x;
        s1 += cs[i] * (double)qv.y;
        s2 += cs[i] * (double)qv.z;
        s3 += cs[i] * (double)qv.w;
      }
      v2d wa = *reinterpret_cast<const v2d*>(&pr.w[n]);
      v2d wb = *reinterpret_cast<const v2d*>(&pr.w[n + 2]);
      wa.x -= s0;
      wa.y -= s1;
      wb.x -= s2;
      wb.y -= s3;
      *reinterpret_cast<v2d*>(&pr.w[n]) = wa;
      *reinterpret_cast<v2d*>(&pr.w[n + 2]) = wb;
      nrm += wa.x * wa.x + wa.y * wa.y + wb.x * wb.x + wb.y * wb.y;
    }
  }
  nrm = block_sum(nrm, sh);
  if (t == 0) partial[((int64_t)p * kmax) * kLzBlocks + b] = nrm;
}

// Number of eigenvalues of the tridiagonal (a, b) below x (Sturm sequence).
__device__ int sturm_count(const double* a, const double* b, int k, double x, double pivmin) {
  int cnt = 0;
  double d = a[0] - x;
  if (fabs(d) < pivmin) d = -pivmin;
  cnt += d < 0.0;
  for (int i = 1; i < k; ++i) {
    d = (a[i] - x) - b[i - 1] * b[i - 1] / d;
    if (fabs(d) < pivmin) d = -pivmin;
    cnt += d < 0.0;
  }
  return cnt;
}

// Lowest eigenpair of T_{j+1}, stop test, advance.  One wave per problem.
// Eigenvalue: multisection with Sturm counts (64 points per round).
// Eigenvector: inverse iteration with the shift just below the eigenvalue,
// where T - sigma I is positive definite and its LDL^T needs no pivoting.
__global__ __launch_bounds__(64) void k_tridiag(LzCtrl* ctrl, int32_t* active, const double* alpha, double* beta,
                                                double* ritz, int kmax, double tol_E, double tol_res,
                                                double tol_first, double rel_first) {
  __shared__ double a[1024], b[1024], dd[1024], ll[1024], y[1024];
  __shared__ double s_lo, s_hi;
  const int p = blockIdx.x;
  if (!active[p]) return;
  const int lane = threadIdx.x;
  const int j = ctrl[p].j;
  const int k = j + 1;
  const double bnew = ctrl[p].beta_j;
  for (int i = lane; i < k; i += 64) {
    a[i] = alpha[(int64_t)p * kmax + i];
    b[i] = i < k - 1 ? beta[(int64_t)p * kmax + i] : 0.0;
  }
  __syncthreads();
  // Gershgorin interval
  double lo = 1e300, hi = -1e300, bmax = 0.0;
  for (int i = lane; i < k; i += 64) {
    const double r = (i > 0 ? fabs(b[i - 1]) : 0.0) + (i < k - 1 ? fabs(b[i]) : 0.0);
    lo = fmin(lo, a[i] - r);
    hi = fmax(hi, a[i] + r);
    if (i < k - 1) bmax = fmax(bmax, fabs(b[i]));
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o, 64));
    hi = fmax(hi, __shfl_xor(hi, o, 64));
    bmax = fmax(bmax, __shfl_xor(bmax, o, 64));
  }
  const double pivmin = fmax(1e-300, 1e-290 * bmax * bmax);
  double theta;
  if (k == 1) {
    theta = a[0];
  } else {
    const double pad = 1e-14 * fmax(fabs(lo), fabs(hi)) + 1e-300;
    lo -= pad;
    hi += pad;
    for (int round = 0; round < 40; ++round) {
      const double x = lo + (hi - lo) * (double)(lane + 1) / 65.0;
      const int c = sturm_count(a, b, k, x, pivmin);
      const unsigned long long m = __ballot(c >= 1);
      // first lane whose point has at least one eigenvalue below it
      int first = m ? __ffsll((long long)m) - 1 : 64;
      const double nlo = first == 0 ? lo : lo + (hi - lo) * (double)first / 65.0;
      const double nhi = first == 64 ? hi : lo + (hi - lo) * (double)(first + 1) / 65.0;
      lo = nlo;
      hi = nhi;
      if (hi - lo <= 2.5e-16 * fmax(fabs(lo), fabs(hi)) + pivmin) break;
    }
    theta = 0.5 * (lo + hi);
  }
  if (lane == 0) {
    if (k == 1) {
      y[0] = 1.0;
    } else {
      const double sigma = theta - (1e-10 * fabs(theta) + 1e-13 * (fabs(lo) + fabs(hi)) + 1e-300);
      dd[0] = a[0] - sigma;
      for (int i = 1; i < k; ++i) {
        ll[i] = b[i - 1] / dd[i - 1];
        dd[i] = (a[i] - sigma) - ll[i] * b[i - 1];
      }
      for (int i = 0; i < k; ++i) y[i] = 1.0;
      for (int it = 0; it < 4; ++it) {
        for (int i = 1; i < k; ++i) y[i] -= ll[i] * y[i - 1];     // L z = y
        for (int i = 0; i < k; ++i) y[i] /= dd[i];                // D
        for (int i = k - 2; i >= 0; --i) y[i] -= ll[i + 1] * y[i + 1];  // L^T
        double nrm = 0.0;
        for (int i = 0; i < k; ++i) nrm += y[i] * y[i];
        nrm = 1.0 / sqrt(nrm);
        for (int i = 0; i < k; ++i) y[i] *= nrm;
      }
    }
    if (y[0] < 0.0)
      for (int i = 0; i < k; ++i) y[i] = -y[i];
    LzCtrl& c = ctrl[p];
    const double res = bnew * fabs(y[k - 1]);
    const bool have_prev = k > 1;
    // rel_first > 0 (a refinement pass): stop once the residual estimate is
    // rel_first times the exact residual beta_0 of the pass's start vector.
    const bool stop_dtheta = rel_first > 0.0
                                 ? (have_prev && res <= rel_first * beta[(int64_t)p * kmax])
                                 : (have_prev && fabs(theta - c.theta_prev) <= tol_E && res <= tol_res);
    // tol_first > 0: the first step used an FP64 matvec, so alpha_0 is the exact
    // Rayleigh quotient of the start vector and beta_0 its exact residual norm.
    const bool stop_first = k == 1 && tol_first > 0.0 && bnew <= tol_first;
    const bool stop_inv = bnew <= 1e-14 * fabs(theta) || stop_first;
    c.theta = theta;
    for (int i = 0; i < k; ++i) ritz[(int64_t)p * kmax + i] = y[i];
    if (stop_dtheta || stop_inv || k >= c.kcap) {
      c.active = 0;
      active[p] = 0;
      c.iters = k;
      c.converged = (stop_dtheta || stop_inv) ? 1 : 0;
      c.flags |= stop_inv ? 1 : 0;
      c.residual = res;
      c.overlap0 = fabs(y[0]);
    } else {
      beta[(int64_t)p * kmax + j] = bnew;
      c.theta_prev = theta;
      c.j = k;
    }
  }
}

// Q[j] = v = w / beta_{j-1}  (j already advanced)
__global__ __launch_bounds__(TB) void k_next(const LzProblem* probs, const LzCtrl* ctrl, const int32_t* active,
                                             const double* beta, int kmax) {
  const int p = blockIdx.y;
  if (!active[p]) return;
  const LzProblem pr = probs[p];
  const int j = ctrl[p].j;
  const double inv = 1.0 / beta[(int64_t)p * kmax + j - 1];
  if (pr.Qf) {
    // the FP32 row, and v = exactly the stored row, so the next matvec acts on the basis vector
    float* q = pr.Qf + (int64_t)(j - 1) * pr.ld;
    for (int64_t n = blockIdx.x * (int64_t)TB + threadIdx.x; n < pr.ld; n += (int64_t)gridDim.x * TB) {
      const float x = (float)(pr.w[n] * inv);
      q[n] = x;
      pr.v[n] = (double)x;
    }
    return;
  }
  double* q = pr.Q + (int64_t)j * pr.ld;
  for (int64_t n = blockIdx.x * (int64_t)TB + threadIdx.x; n < pr.ld; n += (int64_t)gridDim.x * TB) {
    const double x = pr.w[n] * inv;
    q[n] = x;
    pr.v[n] = x;
  }
}

// psi = sum_{i < iters} y_i Q[i]
__global__ __launch_bounds__(TB) void k_ritz(const LzProblem* probs, const LzCtrl* ctrl, const double* ritz, int kmax) {
  const int p = blockIdx.y;
  if (ctrl[p].kcap == 0) return;
  const LzProblem pr = probs[p];
  const int k = ctrl[p].iters;
  const double* y = ritz + (int64_t)p * kmax;
  for (int64_t n = blockIdx.x * (int64_t)TB + threadIdx.x; n < pr.N; n += (int64_t)gridDim.x * TB) {
    double s = 0.0;
    if (pr.Qf) {
      s = y[0] * pr.Q[n];
      for (int i = 1; i < k; ++i) s += y[i] * (double)pr.Qf[(int64_t)(i - 1) * pr.ld + n];
    } else {
      for (int i = 0; i < k; ++i) s += y[i] * pr.Q[(int64_t)i * pr.ld + n];
    }
    pr.psi[n] = s;
  }
}

// psi /= norm0 ; v = psi (input of the residual matvec)
__global__ __launch_bounds__(TB) void k_normalize_psi(const LzProblem* probs, const LzCtrl* ctrl) {
  const int p = blockIdx.y;
  if (ctrl[p].kcap == 0) return;
  const LzProblem pr = probs[p];
  const double inv = 1.0 / ctrl[p].norm0;
  for (int64_t n = blockIdx.x * (int64_t)TB + threadIdx.x; n < pr.N; n += (int64_t)gridDim.x * TB) {
    const double x = pr.psi[n] * inv;
    pr.psi[n] = x;
    pr.v[n] = x;
  }
}

// partial[p][0][b] = sum |w - theta psi|^2
__global__ __launch_bounds__(TB) void k_residual_partial(const LzProblem* probs, const LzCtrl* ctrl, double* partial,
                                                         int kmax) {
  __shared__ double sh[TB];
  const int p = blockIdx.y, b = blockIdx.x;
  const LzProblem pr = probs[p];
  const double th = ctrl[p].theta;
  int64_t lo, hi;
  range_of(pr.N, b, lo, hi);
  double acc = 0.0;
  for (int64_t n = lo + threadIdx.x; n < hi; n += TB) {
    const double r = pr.w[n] - th * pr.psi[n];
    acc += r * r;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[((int64_t)p * kmax) * kLzBlocks + b] = acc;
}

dim3 vec_grid(int P) { return dim3(512, P); }

}  // namespace

void lz_init(int P, const LzProblem* probs, LzCtrl* ctrl, double* partial, int kmax, hipStream_t s) {
  hipLaunchKernelGGL(k_dot_partial, dim3(kLzBlocks, P), dim3(TB), 0, s, probs, (const int32_t*)nullptr, 2, 2,
                     partial, kmax);
  hipLaunchKernelGGL(k_finalize, dim3(P), dim3(TB), 0, s, ctrl, (const int32_t*)nullptr, (const double*)partial,
                     (const double*)nullptr, kmax, 2);
  hipLaunchKernelGGL(k_start, vec_grid(P), dim3(TB), 0, s, probs, ctrl);
}

void lz_iteration_tail(int P, const LzProblem* probs, LzCtrl* ctrl, int32_t* active, double* alpha, double* beta,
                       double* ritz, double* coef, double* partial, double* pnorm, int kmax, double tol_E,
                       double tol_res, double tol_first, double rel_first, int cgs2, hipStream_t s) {
  // first Gram-Schmidt pass (shifted; alpha_j, |w| before and after), then the
  // second pass where the first removed most of w
  for (int pass = 0; pass < 2; ++pass) {
    hipLaunchKernelGGL(k_mdot, dim3(kLzBlocks, P), dim3(TB), 0, s, probs, (const LzCtrl*)ctrl,
                       (const int32_t*)active, partial, pnorm, kmax, pass);
    hipLaunchKernelGGL(k_mdot_finalize, dim3(kmax, P), dim3(TB), 0, s, ctrl, (const int32_t*)active,
                       (const double*)partial, coef, alpha, kmax, pass);
    hipLaunchKernelGGL(k_update, dim3(kLzBlocks, P), dim3(TB), 0, s, probs, (const LzCtrl*)ctrl,
                       (const int32_t*)active, (const double*)coef, partial, kmax, pass);
    hipLaunchKernelGGL(k_finalize, dim3(P), dim3(TB), 0, s, ctrl, (const int32_t*)active, (const double*)partial,
                       (const double*)pnorm, kmax, pass == 0 ? 4 : 1, cgs2);
  }
  hipLaunchKernelGGL(k_tridiag, dim3(P), dim3(64), 0, s, ctrl, active, (const double*)alpha, beta, ritz, kmax, tol_E,
                     tol_res, tol_first, rel_first);
  hipLaunchKernelGGL(k_next, vec_grid(P), dim3(TB), 0, s, probs, (const LzCtrl*)ctrl, (const int32_t*)active,
                     (const double*)beta, kmax);
}

void lz_finish(int P, const LzProblem* probs, LzCtrl* ctrl, double* ritz, double* partial, int kmax, hipStream_t s) {
  hipLaunchKernelGGL(k_ritz, vec_grid(P), dim3(TB), 0, s, probs, (const LzCtrl*)ctrl, (const double*)ritz, kmax);
  hipLaunchKernelGGL(k_dot_partial, dim3(kLzBlocks, P), dim3(TB), 0, s, probs, (const int32_t*)nullptr, 2, 2,
                     partial, kmax);
  hipLaunchKernelGGL(k_finalize, dim3(P), dim3(TB), 0, s, ctrl, (const int32_t*)nullptr, (const double*)partial,
                     (const double*)nullptr, kmax, 2);
  hipLaunchKernelGGL(k_normalize_psi, vec_grid(P), dim3(TB), 0, s, probs, (const LzCtrl*)ctrl);
}

void lz_residual(int P, const LzProblem* probs, LzCtrl* ctrl, double* partial, int kmax, hipStream_t s) {
  hipLaunchKernelGGL(k_residual_partial, dim3(kLzBlocks, P), dim3(TB), 0, s, probs, (const LzCtrl*)ctrl, partial,
                     kmax);
  hipLaunchKernelGGL(k_finalize, dim3(P), dim3(TB), 0, s, ctrl, (const int32_t*)nullptr, (const double*)partial,
                     (const double*)nullptr, kmax, 3);
}

void lz_overlap(int P, const LzProblem* probs, LzCtrl* ctrl, double* partial, int kmax, hipStream_t s) {
  hipLaunchKernelGGL(k_dot_partial, dim3(kLzBlocks, P), dim3(TB), 0, s, probs, (const int32_t*)nullptr, 2, 3,
                     partial, kmax);
  hipLaunchKernelGGL(k_finalize, dim3(P), dim3(TB), 0, s, ctrl, (const int32_t*)nullptr, (const double*)partial,
                     (const double*)nullptr, kmax, 5);
}

}  // namespace idmrg
