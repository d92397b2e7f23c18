// Internal declarations of the idmrg library: work-plan records shared by the
// host plan builders and the gfx950 kernels, and the host-side launchers.
//
// Every device operand is addressed as bases[prob * kNumBases + base] + off,
// so one plan (a list of tasks with element offsets) serves any set of buffers
// and any element type (FP64 masters, FP32 copies, packed bf16 hi/lo pairs).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

namespace idmrg {

constexpr int kNumBases = 8;

// C[M x N] (+)= op(A) op(B); A is [M x K] row-major (or [K x M] when transposed),
// B is [K x N] row-major (or [N x K] when transposed).  beta is 0 or 1.
struct GemmTask {
  int32_t M, N, K;
  int32_t lda, ldb, ldc;
  int32_t prob, beta;
  int32_t abase, bbase, cbase;
  int32_t tile0;      // first global tile of this task (exclusive prefix sum)
  int32_t tiles_n;    // tiles along N
  int32_t pad;
  int64_t aoff, boff, coff;
};
// Workgroups are dispatched round-robin over the 8 XCDs.  A GEMM's device task table ends with one more record
// whose first kXcdRanges int32 fields hold s_0 = 0 <= s_1 <= ... <= s_8 = ntiles: XCD x runs tiles [s_x, s_x+1).
constexpr int kXcdRanges = 9;
static_assert(sizeof(GemmTask) >= kXcdRanges * sizeof(int32_t), "XCD ranges must fit in one task record");

// D[rows x cols] = sum_k coef_k * S_k   (S_k[r][c] at off + r*ld + c, or off + c*ld + r if trans)
// In fragment output mode (split-bf16 T3) output (r, c) is element (r0 + r, c0 + c)
// of a fragment-layout matrix at doff with ldd = its k-fragments per row block;
// c0 is a multiple of 8 and the columns up to the next multiple of 8 past cols
// are written as zeros.
struct MixTask {
  int32_t rows, cols, ldd, prob;
  int32_t dbase, nsrc, src0, tile0;
  int32_t tiles_c, r0, c0, pad;
  int64_t doff;
};

struct MixSrc {
  double coef;
  int64_t off;
  int32_t ld, base;
  int32_t trans, pad;
};

// D[r][c] = S[r][colmap[c]] * rowscale[r] * colscale[c]; absent scales are 1.
// rowscale may be replaced by 1/x (0 for x <= floor) when invert_row is set.
struct ScaleTask {
  int32_t rows, cols, lds, ldd;
  int32_t prob, sbase, dbase, rbase;
  int32_t cbase, invert_row, colmap, tile0;   // colmap < 0: identity map
  int32_t tiles_c, pad;
  int64_t soff, doff, roff, coff;
};

// Fragment layout of the split-bf16 GEMM operands.  A matrix Z[R x K] (the
// GEMM's A, or B transposed, so K is the contraction index) is cut into
// fragments of 16 rows x 32 k, zero-padded at the edges; fragment (rb, kb) of
// a matrix with KB = ceil(K/32) k-fragments per row block starts at 32-bit word
// (rb * KB + kb) * kFragWords.  A fragment holds two planes of 256 words (hi
// bf16 parts, then lo parts); in each plane, lane l in 0..63 owns words
// 4l..4l+3, the bf16 values of row l % 16, k = 8 (l / 16) + e for e = 0..7,
// value e in the low (e even) or high (e odd) half of word 4l + e / 2.  This is
// the operand order of one v_mfma_f32_16x16x32_bf16, so a plane is loaded and
// fed to the MFMA without any rearrangement.
constexpr int kFragRows = 16, kFragK = 32, kFragWords = 512;

// Pack of an FP64 block Z[R x K] into columns [kc0, kc0 + 8 nch) of a
// fragment-layout matrix (KB k-fragments per row block, at word doff of
// destination base dbase): Z(r, k) at soff + r * ld + k (trans: soff + k * ld
// + r) in source base sbase goes to column kc0 + k; the 8-wide chunks are
// written whole for rows 0 .. 16 RB - 1, with zeros outside [R x K] (K = 0
// writes zeros only).  kc0 is a multiple of 8.  hi = bf16(float(z)),
// lo = bf16(float(z) - hi), both rounded to nearest even.  The elements
// Z(dr0 + i, dk0 + i), i < dlen, are packed as Z - sig[shift_slot] (a diagonal
// shift; sig is a device array [problem][2] of the left and right shifts).
// If xbase >= 0 the source block is also written as FP32 in its own
// orientation, row-padded: source element at (row i, column j) of the stored
// matrix goes to xoff + i * xld + j of base xbase.
struct PackTask {
  int32_t R, K, ld, trans;
  int32_t prob, sbase, dbase, tile0;
  int32_t RB, KB, kc0, nch;     // RB = ceil(R / 16)
  int32_t dr0, dk0, dlen, xbase;
  int64_t soff, doff;
  int32_t shift_slot, pad2;     // 2 prob (left shift) or 2 prob + 1 (right shift); -1: none
  int64_t xoff;
  int32_t xld, pad;
};

// The diagonal of a square block: elements off + i (ld + 1), i < len, of base `base`.
struct DiagTask {
  int32_t prob, base, len, ld;
  int64_t off;
};

// One-sided Jacobi SVD of M[r x c] (row-major); n = min(r, c), p = max(r, c).
struct SvdTask {
  int32_t r, c, prob, pad;
  int64_t m_off, x_off, g_off, u_off, v_off, s_off;
  int64_t f_off;   // rows read by the singular-value and output kernels (= x_off unless QR-preconditioned)
};
// Elements of the X base that one matrix of min(r, c) = n rows of length p = max(r, c) needs, and where its
// final rows start (relative to its x_off); see bjsvd.hip.
int64_t bj_x_elems(int n, int p);
int64_t bj_f_rel(int n, int p);

// Selection of kept singular values for one problem (all its centre sectors).
struct SelTask {
  int32_t nsec, sec0;       // sectors [sec0, sec0 + nsec) in the sector arrays
  int32_t ncand, cand0;     // candidates [cand0, cand0 + ncand)
  int32_t m_max, prob;
  double lam_floor, deg_rel;
};

// Per-sector record of the selection (device).
struct SelSector {
  int32_t charge, n;        // centre charge, number of singular values
  int32_t cand0, pad;       // offset of its candidates in the candidate arrays
  int64_t s_off;            // singular values in the S workspace
};

// One segment of an environment overlap: sum over i < rows, j < cols of
// L[aoff + i lda + j] R[boff + i ldb + j], with L and R bases 0 and 1 of its item.
struct OverlapSeg {
  int32_t item, rows, cols, lda, ldb, pad;
  int64_t aoff, boff;
};

// ---------------------------------------------------------------- host errors

struct Status {
  int code = 0;
  std::string msg;
};

#define IDMRG_HIP(call)                                                          \
  do {                                                                           \
    hipError_t e_ = (call);                                                      \
    if (e_ != hipSuccess) {                                                      \
      throw ::idmrg::HipFailure(std::string(#call) + ": " + hipGetErrorString(e_)); \
    }                                                                            \
  } while (0)

struct HipFailure {
  std::string what;
  explicit HipFailure(std::string w) : what(std::move(w)) {}
};
struct InvalidArg {
  std::string what;
  explicit InvalidArg(std::string w) : what(std::move(w)) {}
};

// ---------------------------------------------------------------- launchers

enum class Prec { F64 = 0, F32 = 1, BF16X3 = 2 };

// Grouped GEMM over `ntask` tasks with `ntiles` total tiles.  tiling selects the
// output tile: 0 = 64x64, 1 = 128x64, 2 = 64x128, 3 = 128x128, and for BF16X3
// also 4 = 256x128 (eight waves) and 5 = 128x128 (persistent workgroups);
// tile0/tiles_n of the tasks must have been computed for that tile.
// mode: 0 = NN, 1 = NT, 2 = TN.  Element type chosen by prec:
//   F64: double A, B, C;  F32: float A, B, C;
//   BF16X3: A and B^T in the fragment layout (aoff, boff in 32-bit words; mode,
//   lda and ldb are ignored), float C.
// `active` (nullable) holds one flag per problem; tasks of inactive problems exit at once.
void launch_gemm(Prec prec, int mode, const GemmTask* tasks, int ntask, int ntiles, int xmax,
                 void* const* bases, const int32_t* active, hipStream_t s, int tiling = 0);

// Mix over tasks; tin/tout element types: 0 = double, 1 = float, 3 = split-bf16 pairs in the fragment
// layout (output only; tasks carry r0, c0 and ldd = k-fragments per row block), 4 = float sources whose
// non-transposed rows are 16-byte aligned with lengths a multiple of 4 (input only; 4 columns per load).
// Pairs: (0, 0), (1, 1), (0, 1), (4, 1), (4, 3).
void launch_mix(int tin, int tout, const MixTask* tasks, const MixSrc* srcs, int ntask, int ntiles,
                void* const* bases, const int32_t* active, hipStream_t s);

void launch_scale(const ScaleTask* tasks, const int32_t* colmaps, int ntask, int ntiles,
                  double lam_floor, void* const* bases, hipStream_t s);

// Environment overlaps: partial[g] = the sum of segment g (one workgroup each, a
// fixed reduction tree); out[k] = the partials of item k (segments
// [seg0[k], seg0[k + 1])) added in order.
void launch_overlap(const OverlapSeg* segs, int nseg, const int32_t* seg0, int nitem, void* const* bases,
                    double* partial, double* out, hipStream_t s);

// element conversions (n elements): kind 0 double -> float, kind 1 float -> double
void launch_convert(int kind, const void* src, void* dst, int64_t n, hipStream_t s);

// out[t] = sum of the diagonal of DiagTask t (FP64 sources; one workgroup per task).
void launch_diag_sum(const DiagTask* tasks, int ntask, void* const* bases, double* out, hipStream_t s);
// Energy shifts of the low-precision copies from the diagonal sums: tasks [0, nleft) are diagonals of
// the left environment, the rest of the right one.  sig[2p] (left) and sig[2p + 1] (right) = mean of
// problem p's diagonal elements on that side if flags[2p] (flags[2p + 1]) is set, else 0 (summed in
// task order, one thread); shift[t] = the shift of task t's side and problem.
void launch_sigma(const DiagTask* tasks, int ntask, int nleft, const double* sums, const int32_t* flags, int P,
                  double* sig, double* shift, hipStream_t s);
// FP32 copies (bases dst) of FP64 blocks (bases src, same offsets): diagonal of task t = float(src - shift[t]).
void launch_diag_shift_f32(const DiagTask* tasks, int ntask, void* const* src, void* const* dst, const double* shift,
                           hipStream_t s);
// dst[i] = (double)src[i] + (sig[2 prob] + sig[2 prob + 1]) x[i] (n elements; float src, double x and dst).
void launch_convert_add(const float* src, const double* x, const double* sig, int prob, double* dst, int64_t n,
                        hipStream_t s);

// Fragment packs (256 row-chunks of 8 values per tile); sources are read through sbases, results written
// through dbases; sig: the diagonal shifts (see PackTask; may be null if no task has a shift slot).
void launch_pack(const PackTask* tasks, int ntask, int ntiles, void* const* sbases, void* const* dbases,
                 const double* sig, const int32_t* active, hipStream_t s);

// Blocked one-sided Jacobi (bjsvd.hip): all matrices of `svd` at once.
// bases (device): per problem kNumBases pointers, 1 M, 2 X, 3 G, 4 U, 5 V, 6 S; dtasks = the same tasks on
// the device.
// sync() waits for the stream (the host checks the sweep flags once per sweep).
struct BjScratch {
  double tol = 1e-15;        // relative orthogonality of converged rows
  double zero_rel = 1e-15;   // rows with norm <= zero_rel |M|_F are null rows
  int inner_sweeps = 1;      // cap of the sweeps that diagonalise one 64 x 64 pair Gram matrix
  int max_sweeps = 40;       // YC8 kagome at m = 4096 needs up to 29
  int sweeps = 0;            // out: sweeps run
  int converged = 0;         // out: every matrix met the tolerance
  std::vector<int> done_at;  // out: per matrix, the sweep after which it met the tolerance (-1: never)
  // Null-row completion is needed only where a zero-weight state can be kept.
  // If set, called after the sweeps once the singular values are in S (device);
  // it clears complete[m] for every matrix m whose null rows need no
  // completion (they are then returned as zero vectors).  Unset: all complete.
  std::function<void(std::vector<int32_t>& complete)> need_completion;
  int completed = 0;         // out: matrices whose null rows were completed
};
// The host part of bj_svd, prepared before any device work: the round schedule and the other device
// tables (host, to be copied to the device before bj_svd runs) and the bytes of device scratch the
// rounds need.
struct BjPlan {
  int nm = 0;
  std::vector<char> host;
  size_t scratch = 0;
  size_t omats = 0, oflags = 0, othr = 0, ocomp = 0, b_partial = 0, b_q = 0;
  std::vector<size_t> opair, ogram, oapply;
  std::vector<int> npair, ngram, napply;
  // QR preconditioning: per-matrix table, and per panel the row chunks of the trailing update and of the
  // application of the reflectors to all rows
  int nqr = 0, npanel = 0;
  size_t oqr = 0;
  std::vector<size_t> otrail, ofull;
  std::vector<int> ntrail, nfull, vl1, vl2;   // vl: the longest reflector of panel k (which = 1, 2)
};
void bj_prepare(const std::vector<SvdTask>& svd, BjPlan& plan);
// dev: plan.host on the device; work: plan.scratch bytes of device memory.
void bj_svd(const BjPlan& plan, void* const* dbases, const SvdTask* dtasks, BjScratch& scr, hipStream_t s,
            const char* dev, char* work, const std::function<void()>& sync);
// flag[0] = 1 if any of x[0..n) is NaN or infinite; the caller clears the flag first.
void launch_check_finite(const double* x, int64_t n, int32_t* flag, hipStream_t s);
void launch_select(const SelTask* tasks, int ntask, const SelSector* secs, const double* S,
                   int32_t* kept_per_sec, int32_t* colmap, double* lam_sel, double* scal,
                   hipStream_t s);

// Lanczos vector kernels (batched over problems), see lanczos.hip
struct LzProblem {
  int64_t N;        // elements of the two-site state
  int64_t ld;       // padded length (multiple of kLzAlign): row stride of Q, length of w and v
  double* Q;        // [kcap x ld], zero beyond N in every row
  double* w;        // [ld] matvec output / work vector, zero beyond N
  double* v;        // [ld] current vector (matvec input), zero beyond N
  double* psi;      // [N] caller's vector
  double* s0;       // [ld] normalised start vector (mixed precision only; else null)
  float* Qf;        // FP32 basis: rows 1.. of the basis, row i at Qf + (i - 1) ld (row 0 stays FP64 in Q);
                    // null: every row in Q
};

struct LzCtrl {     // device, one per problem
  int32_t j;        // index of the current Lanczos vector
  int32_t active;
  int32_t iters;
  int32_t converged;
  int32_t flags;
  int32_t kcap;
  int32_t reorth;   // this iteration needs the second Gram-Schmidt pass
  int32_t reorths;  // second passes so far
  double theta, theta_prev, beta_j, residual, norm0, overlap0, ynorm;
  double shift;     // sigma: from iteration 1 on, H - sigma I is orthogonalised (sigma = alpha_0)
};

constexpr int kLzBlocks = 512;   // partial-sum blocks per problem
constexpr int kLzAlign = 256;    // padding unit of the Lanczos vectors (elements)
constexpr int kLzMaxK = 1024;    // upper bound of k_max (tridiagonal kept in LDS)

// ctrl[] and active[] are initialised by the host before lz_init.
void lz_init(int P, const LzProblem* probs, LzCtrl* ctrl, double* partial, int kmax, hipStream_t s);
// pnorm: [P][kLzBlocks] partial sums of the norm before orthogonalisation.
void lz_iteration_tail(int P, const LzProblem* probs, LzCtrl* ctrl, int32_t* active, double* alpha, double* beta,
                       double* ritz, double* coef, double* partial, double* pnorm, int kmax, double tol_E,
                       double tol_res, double tol_first, double rel_first, int cgs2, hipStream_t s);
void lz_finish(int P, const LzProblem* probs, LzCtrl* ctrl, double* ritz, double* partial, int kmax, hipStream_t s);
void lz_residual(int P, const LzProblem* probs, LzCtrl* ctrl, double* partial, int kmax, hipStream_t s);
// ctrl.overlap0 = |<s0, psi>| (psi normalised by lz_finish, s0 the normalised start vector)
void lz_overlap(int P, const LzProblem* probs, LzCtrl* ctrl, double* partial, int kmax, hipStream_t s);

}  // namespace idmrg
