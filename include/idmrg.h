/*
 * idmrg.h -- C-ABI of the MI355X (gfx950) hot path of the parallel
 * infinite-size DMRG of H. Ueda, "Infinite-Size Density Matrix
 * Renormalization Group with Parallel Hida's Algorithm" (arXiv 1606.06790).
 *
 * Five calls follow the paper's statement of the per-superblock problem:
 *   heff_apply            apply the superblock Hamiltonian H^(n)_i
 *                         (Sec. 2, Step 3; Fig. 2(b))
 *   lanczos_solve_batch   solve H^(n)_i Psi = e Psi from a start vector for
 *                         the l/2 superblocks of one iteration (Steps 3, 3')
 *   truncate_twosite      Psi = U Lambda V^dagger and keep the largest states
 *                         (Steps 4, 6; Eqs. (13), (14))
 *   update_env            block-spin transformation of the expanded blocks
 *                         (Step 6, Eqs. (4), (5), with Step 2' folded in)
 *   predict_wavefunction  start vector of the next iteration (Eq. (10))
 * Two more serve the uniform MPS the iteration converges to (Eq. (11)) and its
 * observables (Sec. 4): twosite_to_right_iso (a two-site piece as the right
 * isometry of its fused site) and env_overlap (expectation values as the
 * contraction of a left and a right environment).
 * Every call is batch-first: it takes nprob >= 1 independent problems and
 * runs them in one set of grouped launches.
 *
 * ---------------------------------------------------------------------------
 * Data conventions (all floating point data is IEEE FP64 unless stated).
 *
 * Charges are 2*S^z (integers) in the left-flux convention: the charge of a
 * bond sector is the total charge of everything to the left of that bond.
 * A dense (no symmetry) problem is the special case where every charge is 0.
 *
 * A leg (idmrg_leg) lists sectors with strictly ascending charge q[k] and
 * dimension dim[k] >= 1.  Local states have charges qp[0..d-1].
 *
 * An MPO tensor W[w][w'][s][s'] (idmrg_mpo) is dense, row-major, on the host,
 * with channel charges ql (rows, the cut to the left of the site) and qr
 * (columns).  W[w][w'][s][s'] may be nonzero only if
 * qp[s] - qp[s'] == qr[w'] - ql[w].  Channel 0 is "complete" and channel D-1
 * is "identity"; W[0][0] and W[dl-1][dr-1] must be the identity (the paper's
 * lower-triangular form whose last row and first column are the boundary
 * vectors, Sec. 2 after Eq. (1)).
 *
 * Device tensors are flat FP64 arrays in these orders (k ascending everywhere):
 *   two-site state Psi[alpha,s1,s2,beta], legs A (alpha), B (beta):
 *       blocks for b in B, a in A, s1, s2 with q_a+qp[s1]+qp[s2] == q_b,
 *       each block [dim_a x dim_b] row-major.
 *   left environment L[alpha,w,alpha'] (leg A, channels = rows of W1):
 *       for a' in A, for w = 0..dl-2, if q_a'+ql[w] is a sector a of A:
 *       block [dim_a x dim_a'] row-major.  Channel dl-1 (identity) is not stored.
 *   right environment R[beta,w,beta'] (leg B, channels = columns of W2):
 *       for b in B, one row-major [dim_b x K_b] matrix whose columns run over
 *       w = 1..dr-1 and the sector b' with q_b' = q_b - qr[w] (if present).
 *       Channel 0 (identity) is not stored.
 *   left isometry U[(alpha,s),gamma] (new leg C):
 *       for c in C, a row-major [r_c x k_c] matrix, rows over a in A, s with
 *       q_a + qp[s] == q_c.
 *   right isometry V[(s,beta),gamma] (new leg C):
 *       for c in C, a row-major [r'_c x k_c] matrix, rows over s, b in B with
 *       q_b - qp[s] == q_c.
 *   singular values lambda: for c in C, k_c values (descending, then zeros).
 *
 * Ownership: the caller allocates every input and output buffer.  Device
 * scratch (intermediates, low-precision operand copies, the Krylov basis, work
 * plans) comes from a workspace: the caller sizes it with
 * idmrg_workspace_size() and attaches it with idmrg_set_workspace(); while one
 * is attached no call allocates device memory.  Without one the library keeps
 * a block of its own, allocated with hipMalloc on first use, grown (after the
 * stream has drained) when a call needs more, and freed by idmrg_destroy.
 * Work plans reach the device through a pinned staging ring allocated by
 * idmrg_create.  The library keeps no pointer to caller memory after a call
 * returns, except the attached workspace.
 *
 * Streams: all device work of a context is enqueued on its stream.  Calls that
 * return host results (lanczos_solve_batch, truncate_twosite) synchronise that
 * stream before returning; heff_apply, update_env and predict_wavefunction are
 * asynchronous (the host waits only if more than the staging ring's 32 MiB of
 * plan uploads are still queued).  Back-to-back calls may share one workspace:
 * their work runs in stream order.
 *
 * Errors: 0 = success; > 0 = warning (IDMRG_WARN_NOCONV); < 0 = error, with a
 * message from idmrg_last_error().  No C++ exception crosses this boundary.
 * Every shape, charge and capacity is validated on the host before any
 * kernel is launched; an invalid argument returns IDMRG_EINVAL and launches
 * nothing.
 */
#ifndef IDMRG_H
#define IDMRG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IDMRG_OK 0
#define IDMRG_WARN_NOCONV 1
#define IDMRG_EINVAL (-1)
#define IDMRG_ENOMEM (-2)
#define IDMRG_EHIP (-3)
#define IDMRG_ENUMERIC (-4)
#define IDMRG_EUNSUPPORTED (-5)

/* arithmetic policies of the H_eff contractions */
#define IDMRG_PREC_F64 0      /* FP64 MFMA */
#define IDMRG_PREC_F32 1      /* operands rounded to FP32, FP32 MFMA, FP32 accumulate */
#define IDMRG_PREC_BF16X3 2   /* operands split a = hi + lo (bf16), hi*hi + hi*lo + lo*hi, FP32 accumulate */

#define IDMRG_LEFT 0
#define IDMRG_RIGHT 1

typedef struct idmrg_ctx idmrg_ctx;

typedef struct {
    int32_t nsec;
    const int32_t* q;    /* host [nsec], strictly ascending */
    const int32_t* dim;  /* host [nsec], each >= 1 */
} idmrg_leg;

typedef struct {
    int32_t dl, dr, d;
    const double* w;     /* host [dl][dr][d][d] */
    const int32_t* ql;   /* host [dl] */
    const int32_t* qr;   /* host [dr] */
    const int32_t* qp;   /* host [d] */
} idmrg_mpo;

/* One superblock Hamiltonian H^(n)_i = {L W1 W2 R} (Sec. 2, Step 3). */
typedef struct {
    idmrg_leg left;           /* alpha leg = leg of L */
    idmrg_leg right;          /* beta leg = leg of R */
    const idmrg_mpo* w1;      /* W_{f(2i+n-1)}: rows = channels of L */
    const idmrg_mpo* w2;      /* W_{f(2i+n)}: columns = channels of R; w1->dr == w2->dl */
    const double* L;          /* device, left-environment layout */
    const double* R;          /* device, right-environment layout */
} idmrg_heff;

/* ------------------------------------------------------------------ context */

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the default stream). */
int idmrg_create(idmrg_ctx** ctx, int device, void* hip_stream);
int idmrg_destroy(idmrg_ctx* ctx);
int idmrg_set_stream(idmrg_ctx* ctx, void* hip_stream);
const char* idmrg_last_error(const idmrg_ctx* ctx);

/* Element counts of the flat layouts above (host only; no device work). */
int64_t idmrg_psi_size(idmrg_leg A, idmrg_leg B, int32_t d, const int32_t* qp);
int64_t idmrg_envL_size(idmrg_leg A, int32_t dl, const int32_t* ql);
int64_t idmrg_envR_size(idmrg_leg B, int32_t dr, const int32_t* qr);
int64_t idmrg_U_size(idmrg_leg A, int32_t d, const int32_t* qp, idmrg_leg C);
int64_t idmrg_V_size(idmrg_leg B, int32_t d, const int32_t* qp, idmrg_leg C);

/* Algorithmic work of one heff_apply of H (host only): flops of the two
 * environment GEMM stages plus the W mixing, counted from the block lists
 * (identity channels and symmetry-forbidden blocks excluded), and the bytes
 * that the matvec must move at least once (environments, input, output). */
int idmrg_heff_work(const idmrg_heff* H, double* flops, double* bytes);

/* Profiling: when enabled, every launch of the library is bracketed by HIP
 * events on the context stream.  idmrg_profile_get() synchronises the stream
 * and returns, for one kernel class, the number of launches, their summed
 * duration (ms) and their summed algorithmic flops (FP64-equivalent
 * multiply-adds x 2).  Classes: 0 H_eff GEMM stage 1, 1 H_eff GEMM stage 2,
 * 2 H_eff mixing (0-2 with FP64 arithmetic), 3 precision conversions,
 * 4 Lanczos vector kernels, 5 SVD, 6 truncation gather/select/scatter,
 * 7 environment update, 8 prediction, 9 H_eff GEMM stage 1, 10 H_eff GEMM
 * stage 2, 11 H_eff mixing (9-11 with FP32 or split-bf16 arithmetic).
 * idmrg_profile(ctx, 1) also clears the counters. */
#define IDMRG_PROF_CLASSES 12
int idmrg_profile(idmrg_ctx* ctx, int enable);
int idmrg_profile_get(idmrg_ctx* ctx, int cls, int64_t* launches, double* ms, double* flops);

/* ------------------------------------------------------------------ calls */

/* y_p = H_p x_p for p < nprob (Sec. 2, Step 3; Fig. 2(b)):
 *   y[a,s1,s2,b] = sum L[a,w,a'] W1[w,w',s1,t1] W2[w',w'',s2,t2] R[b,w'',b'] x[a',t1,t2,b'].
 * x[p], y[p]: device pointers (host array of nprob pointers) in the Psi
 * layout of H[p].left/right; x and y must not overlap.  prec selects the
 * arithmetic (IDMRG_PREC_*); FP64 inputs and outputs in every case. */
int heff_apply(idmrg_ctx* ctx, int nprob, const idmrg_heff* H,
               const double* const* x, double* const* y, int prec);

/* heff_apply for callers that cannot allocate memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * plan and kernels as heff_apply, bitwise the same results, but the scratch is
 * a file-scope device array of 64 MiB (one per GPU, set up by idmrg_create and
 * held until the process ends) instead of the workspace, and the call makes
 * no device or pinned allocation.  Calls whose scratch (idmrg_workspace_size
 * with IDMRG_OP_HEFF) exceeds 64 MiB return IDMRG_EINVAL and launch nothing.
 * Every call on one GPU, from any context or stream, shares that array: calls
 * that overlap in time on one GPU race.  Asynchronous like heff_apply. */
int heff_apply_static(idmrg_ctx* ctx, int nprob, const idmrg_heff* H,
                      const double* const* x, double* const* y, int prec);

typedef struct {
    double tol_E;       /* stop when |theta_k - theta_{k-1}| <= tol_E ... */
    double tol_res;     /* ... and the residual estimate beta_k |y_k| <= tol_res */
    int32_t k_max;      /* at most min(k_max, N) Lanczos vectors */
    int32_t prec;       /* IDMRG_PREC_* of the matvec inside the iteration */
    int32_t chunk;      /* iterations between host checks of the device stop flags */
    int32_t fp32_basis; /* mixed precision only: 1 stores the Krylov vectors of the first pass, after its
                           start vector, in FP32 (half the bytes of that pass's re-orthogonalisation; every
                           sum stays FP64, and the refinement passes keep an FP64 basis); 0 keeps every
                           vector FP64.  Ignored for IDMRG_PREC_F64. */
    int32_t cgs2;       /* 1: second Gram-Schmidt pass in every iteration (classical CGS2);
                           0: only where the first pass removes more than 99 % of |w|^2 */
    int32_t graph;      /* 1: once the GEMM tilings are tuned, every full chunk of iterations
                           is captured into a HIP graph (one per pass shape, on a capture
                           stream owned by the context) and replayed on the context stream;
                           the same kernels in the same order, so results are bitwise those
                           of 0 (direct launches).  Ignored while profiling is enabled. */
} idmrg_lanczos_opts;

typedef struct {
    int32_t iters;        /* Lanczos vectors used (k) */
    int32_t converged;    /* 1 if a stop rule other than k = k_max fired */
    int32_t fp64_matvecs; /* FP64 matvecs of the refinement (mixed precision) */
    int32_t flags;        /* bit 0: invariant subspace (beta ~ 0) */
    int32_t reorth_passes; /* iterations that needed the second Gram-Schmidt pass */
    int32_t reserved;
    double residual;      /* |H psi - e psi| (FP64 matvec) after the solve */
    double overlap0;      /* |<start/|start|, psi>|, so 1 - overlap0 is the fidelity error of Eq. (12) */
} idmrg_lanczos_info;

/* Lowest eigenpair of each H_p by Lanczos with full FP64 re-orthogonalisation
 * (classical Gram-Schmidt against the whole basis every iteration, after a
 * shift by the first Rayleigh quotient; a second pass where the first removed
 * more than 99 % of the vector's norm squared), FP64 tridiagonal eigensolver
 * and Ritz vector, all on the device (Step 3; Step 3' for the start vector).
 * psi[p]: device, in: start vector (any nonzero norm), out: normalised ground
 * state.  energy[p], info[p]: host outputs.  Synchronises the stream.
 * Returns IDMRG_WARN_NOCONV if any problem stopped at k = k_max. */
int lanczos_solve_batch(idmrg_ctx* ctx, int nprob, const idmrg_heff* H, double* const* psi,
                        const idmrg_lanczos_opts* opts, double* energy, idmrg_lanczos_info* info);

typedef struct {
    /* inputs */
    idmrg_leg left, right;     /* legs of psi */
    const double* psi;         /* device, normalised two-site state */
    int32_t cap_sec;           /* capacity of q_out/dim_out */
    int32_t* q_out;            /* host out: new leg charges */
    int32_t* dim_out;          /* host out: new leg dims */
    double* U;                 /* device out, U layout of the new leg; capacity cap_U doubles */
    double* V;                 /* device out, V layout; capacity cap_V doubles */
    double* lambda;            /* device out; capacity cap_lam doubles */
    int64_t cap_U, cap_V, cap_lam;
    /* outputs */
    int32_t nsec_out;
    int32_t m_kept;
    double eps;                /* discarded weight, Eq. (14) */
    double eps_prime;          /* best fidelity error, Eq. (13) */
    double cut_gap;            /* relative gap at the cut (-1 if no nonzero value was cut) */
    int32_t svd_sweeps;        /* Jacobi sweeps run (the same for every problem of the call) */
    int32_t svd_converged;     /* 1 if every block met the orthogonality tolerance */
    int32_t null_completed;    /* 1 if the null-row completion ran for this problem's blocks */
    int32_t reserved;
} idmrg_trunc;

/* Psi = U Lambda V^dagger per centre charge (FP64 one-sided Jacobi SVD on the
 * device), keep the largest min(m_max, ...) states (Steps 4, 6).  Readings:
 * values <= lam_floor count as zero; zero-weight states are kept (in
 * ascending charge order) only when every candidate state is kept, so that the
 * kept space never depends on which null vectors the decomposition found;
 * otherwise at most the nonzero values are kept (m_kept may then be below
 * m_max); the cut is moved up past values within deg_rel (relative) of the
 * last kept one.
 * lambda is normalised over the full spectrum (sum lambda^2 = 1) and the
 * kept values are not renormalised.  Singular vectors of values at most
 * min(max(lam_floor, 1e-15), 1e-14) times their block's Frobenius norm are replaced by an
 * orthonormal completion (they carry no reliable direction), so U and V are
 * isometries to rounding in every case.  The completion runs only for problems
 * where the selection can keep such a vector; elsewhere they are never kept.
 * Rows count as orthogonal at |<x_i, x_j>| <= max(1e-15, 4.4e-16 sqrt(p)) |x_i| |x_j|
 * with p the longest row length among all blocks of the call, so a problem's
 * result can differ at that level between a batched and a single call.
 * Synchronises the stream.  Returns
 * IDMRG_WARN_NOCONV if the Jacobi sweeps did not converge (the result is
 * still written and svd_converged is 0), and IDMRG_ENUMERIC (nothing written)
 * if psi holds a NaN or an infinity. */
int truncate_twosite(idmrg_ctx* ctx, int nprob, int32_t d, const int32_t* qp, int32_t m_max,
                     double lam_floor, double deg_rel, idmrg_trunc* t);

typedef struct {
    idmrg_leg old_leg;         /* leg of env_old (alpha for LEFT, beta for RIGHT) */
    idmrg_leg new_leg;         /* leg of the isometry's new index */
    const idmrg_mpo* w;        /* W1 (LEFT: rows = channels of env_old) or W2 (RIGHT: columns) */
    const double* env_old;     /* device */
    const double* iso;         /* device: U (LEFT) or V (RIGHT) */
    double* env_new;           /* device out: L layout with channels = columns of W (LEFT),
                                  R layout with channels = rows of W (RIGHT) */
} idmrg_env_update;

/* Block-spin transformation (Step 6):
 *   LEFT  (Eq. (4)): L'[w'](c,c') = sum u[(a,s),c] L[w](a,a') W[w,w',s,s'] u[(a',s'),c']
 *   RIGHT (Eq. (5)): R'[w](c,c') = sum v[(s,b),c] W[w,w'',s,s'] R[w''](b,b') v[(s',b'),c']
 * Environments stay FP64 in every mode. */
int update_env(idmrg_ctx* ctx, int nprob, int side, const idmrg_env_update* u);

typedef struct {
    idmrg_leg leg_a;           /* leg of lam_i = alpha leg of the prediction */
    idmrg_leg leg_beta;        /* leg of lam_prev = the contracted index */
    idmrg_leg leg_b;           /* leg of lam_ip1 = beta leg of the prediction */
    const double* lam_i;       /* device: lambda^(n-1)_i */
    const double* V_i;         /* device: V^(n-1)_i, V layout (B = leg_beta, C = leg_a) */
    const double* lam_prev;    /* device: lambda^(n-2)_{i+1} */
    const double* U_ip1;       /* device: U^(n-1)_{i+1}, U layout (A = leg_beta, C = leg_b) */
    const double* lam_ip1;     /* device: lambda^(n-1)_{i+1} */
    double* psi;               /* device out: Psi layout with legs (leg_a, leg_b) */
} idmrg_predict;

/* Eq. (10): psi[a,s,s',a'] = sum_b lam_i[a] v_i[(s,b),a] u~[b,s',a'],
 *           u~[b,s',a'] = u_{i+1}[(b,s'),a'] lam_ip1[a'] / lam_prev[b] (0 if lam_prev[b] <= lam_floor). */
int predict_wavefunction(idmrg_ctx* ctx, int nprob, int32_t d, const int32_t* qp, double lam_floor,
                         const idmrg_predict* p);

/* ------------------------------------------------------------------ uniform MPS */

/* Sec. 3, Eq. (11): after iteration n the wavefunction repeats a unit cell of
 * the two-site pieces B_i = V^(n)dagger_i U~^(n)_{i+1}, which are the Eq. (10)
 * states of predict_wavefunction with lam_i = 1.  A two-site state in the
 * Psi layout with legs (A, B) is, unchanged, the left isometry U of one fused
 * site (s = s1 d + s2, charge qp[s1] + qp[s2]) with new leg B, so update_env
 * (LEFT) applies the left transfer matrix of a piece, with an MPO of the fused
 * site carrying operators (Sec. 4: bond strengths, correlations).  The right
 * transfer matrix needs the piece as the right isometry V of the fused site,
 * which twosite_to_right_iso writes. */
typedef struct {
    idmrg_leg left;            /* A */
    idmrg_leg right;           /* B */
    const double* psi;         /* device: Psi layout with legs (A, B) */
    double* out;               /* device out: V layout of the fused site (B, fused qp, C = A) */
} idmrg_twosite_item;

/* out = psi read as V[(s, b), a] = psi[a, s1, s2, b], s = s1 d + s2: every
 * block of psi transposed into its place in the V layout of the fused site
 * (local charges qp[s1] + qp[s2] for s = s1 d + s2, d = the d of qp).  An
 * exact copy; asynchronous on the context stream. */
int twosite_to_right_iso(idmrg_ctx* ctx, int nitem, int32_t d, const int32_t* qp, const idmrg_twosite_item* items);

typedef struct {
    idmrg_leg leg;             /* the bond both environments live on */
    int32_t nl;                /* channels of L (its W's columns, incl. the unstored identity) */
    const int32_t* ql;         /* host [nl]: channel charges of L */
    const double* L;           /* device: left-environment layout on leg with charges ql */
    int32_t nr;                /* channels of R (incl. the unstored identity channel 0) */
    const int32_t* qr;         /* host [nr]: channel charges of R */
    const double* R;           /* device: right-environment layout on leg with charges qr */
    int32_t wl, wr;            /* stored channels to contract: 0 <= wl < nl - 1, 1 <= wr < nr, ql[wl] == qr[wr] */
} idmrg_overlap_item;

/* Sec. 4, expectation values of the uniform MPS: out[k] (host) = sum over a, a'
 * of L[a, wl, a'] R[a, wr, a'] for item k (the contraction of a left and a
 * right environment across one bond).  Deterministic order; synchronises the
 * context stream.  IDMRG_ENUMERIC if a result is not finite. */
int env_overlap(idmrg_ctx* ctx, int nitem, const idmrg_overlap_item* items, double* out);

/* ------------------------------------------------------------------ workspace */

/* Operations for idmrg_workspace_size. */
#define IDMRG_OP_HEFF 0       /* heff_apply;            desc: idmrg_heff[nprob]       */
#define IDMRG_OP_LANCZOS 1    /* lanczos_solve_batch;   desc: idmrg_heff[nprob]       */
#define IDMRG_OP_TRUNCATE 2   /* truncate_twosite;      desc: idmrg_trunc[nprob]      */
#define IDMRG_OP_ENV_LEFT 3   /* update_env(LEFT);      desc: idmrg_env_update[nprob] */
#define IDMRG_OP_ENV_RIGHT 4  /* update_env(RIGHT);     desc: idmrg_env_update[nprob] */
#define IDMRG_OP_PREDICT 5    /* predict_wavefunction;  desc: idmrg_predict[nprob]    */
#define IDMRG_OP_TWOSITE_V 6  /* twosite_to_right_iso;  desc: idmrg_twosite_item[nprob] */
#define IDMRG_OP_OVERLAP 7    /* env_overlap;           desc: idmrg_overlap_item[nprob] */

/* The scalar arguments of the call being sized (unused fields are ignored). */
typedef struct {
    int32_t prec;                     /* IDMRG_OP_HEFF: its prec argument */
    int32_t m_max;                    /* IDMRG_OP_TRUNCATE */
    int32_t d;                        /* IDMRG_OP_TRUNCATE, IDMRG_OP_PREDICT: local dimension ... */
    int32_t pad;
    const int32_t* qp;                /* ... and local charges */
    const idmrg_lanczos_opts* opts;   /* IDMRG_OP_LANCZOS: its options (k_max, prec) */
} idmrg_ws_query;

/* Bytes of device workspace that the call `op` with these nprob descriptors
 * needs (host work only: the call's plan is built, validated and kept, so that
 * the call itself, made next with the same shapes, does not build it again).
 * Depends on the legs, MPO tensors and options, not on device pointers or
 * values.  Errors: IDMRG_EINVAL for invalid descriptors. */
int idmrg_workspace_size(idmrg_ctx* ctx, int op, int nprob, const void* desc, const idmrg_ws_query* q,
                         size_t* bytes);

/* Attach a caller-owned device buffer (256-byte aligned, on the context's
 * device, at least the size idmrg_workspace_size reports for every call that
 * will use it) as the scratch of every later call, or detach with ptr = NULL
 * (the library then allocates its own again).  Attaching frees the library's
 * own block.  A call that needs more than the attached bytes returns
 * IDMRG_ENOMEM without launching anything; calls never allocate device memory
 * while a workspace is attached.  The caller must keep the buffer alive until
 * the work queued on the context stream that uses it has run. */
int idmrg_set_workspace(idmrg_ctx* ctx, void* ptr, size_t bytes);

/* The GEMM tile autotuner.  The first matvecs of a Lanczos call whose stage
 * shapes fall in a bucket not yet measured each run one tiling (the results do
 * not depend on it) and the fastest is kept for that bucket: precision, stage
 * (0: environment-L GEMM, 1: environment-R GEMM), log2 of the stage's flops and
 * of its flop-weighted mean N and K.  Tilings: 0 64x64, 1 128x64, 2 64x128,
 * 3 128x128, 4 256x128 (split-bf16 only: eight waves, the operand reads of
 * each K-slab overlapped with the previous slab's MFMAs), 5 128x128 (split-bf16
 * only: persistent workgroups that copy the next tile's first K-slab while the
 * current tile finishes).  idmrg_tune_get copies up
 * to cap entries (with the trial times, -1 where a tiling was not tried) and
 * sets *n to the number of entries; idmrg_tune_set installs entries (a cache
 * from an earlier process), which are then not measured again. */
#define IDMRG_TUNE_VARIANTS 8
typedef struct {
    int32_t prec, stage, log2_flops, log2_n, log2_k, tiling;
    float trial_ms[IDMRG_TUNE_VARIANTS];
} idmrg_tune_entry;
int idmrg_tune_get(idmrg_ctx* ctx, idmrg_tune_entry* out, int cap, int* n);
int idmrg_tune_set(idmrg_ctx* ctx, const idmrg_tune_entry* in, int n);

/* Counters of a context since idmrg_create. */
typedef struct {
    int64_t device_allocs;   /* hipMalloc calls for the library's own scratch block */
    int64_t stream_syncs;    /* synchronisations of the context stream made by the library */
    int64_t staged_bytes;    /* bytes of work plans copied to the device */
    int64_t plan_builds;     /* work plans built (a size query and the call that follows it build one) */
} idmrg_stats;
int idmrg_get_stats(idmrg_ctx* ctx, idmrg_stats* out);

#ifdef __cplusplus
}
#endif
#endif /* IDMRG_H */
