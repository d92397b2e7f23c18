// Host-side layouts and work-plan builders (no device code).
//
// Each builder turns the block structure of one problem into task lists for
// the grouped kernels; element offsets are relative to the problem's base
// pointers (see internal.h), so a plan is independent of the buffers it runs on.
#pragma once

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "idmrg.h"
#include "internal.h"

namespace idmrg {

struct Leg {
  std::vector<int> q, dim;
  int n() const { return (int)q.size(); }
  int find(int charge) const;   // sector index or -1
  int64_t total() const;
};

struct Mpo {
  int dl = 0, dr = 0, d = 0;
  std::vector<double> w;        // [dl][dr][d][d]
  std::vector<int> ql, qr, qp;
  double at(int a, int b, int s, int t) const { return w[(((int64_t)a * dr + b) * d + s) * d + t]; }
};

Leg make_leg(const idmrg_leg& l, const char* what);
Mpo make_mpo(const idmrg_mpo* m, const char* what);
std::vector<int> make_qp(int d, const int32_t* qp);

// ---- layouts (element counts and offsets of the flat formats in idmrg.h)

struct PsiLayout {
  struct Blk { int b, a, s1, s2; int64_t off; int da, db; };
  std::vector<Blk> blk;
  std::map<long long, int> index;   // key(a, s1, s2) -> block
  std::vector<int64_t> b_first;     // first element of the blocks with right sector b (-1 if none)
  std::vector<int> b_rows;          // rows of the stacked matrix of right sector b
  int64_t size = 0;
  static long long key(int a, int s1, int s2) { return ((long long)a * 64 + s1) * 64 + s2; }
  int find(int a, int s1, int s2) const {
    auto it = index.find(key(a, s1, s2));
    return it == index.end() ? -1 : it->second;
  }
};
PsiLayout psi_layout(const Leg& A, const Leg& B, const std::vector<int>& qp);

struct EnvLLayout {       // L[alpha, w, alpha'] without the identity channel (last)
  std::vector<int64_t> stack_off;          // per column sector a'
  std::vector<int> rows;                   // stacked rows M_a'
  std::vector<std::vector<int>> row_off;   // [a'][w] row offset inside the stack, -1 if absent
  std::vector<std::vector<int>> a_out;     // [a'][w] row sector
  int64_t size = 0;
};
EnvLLayout envL_layout(const Leg& A, const std::vector<int>& dq);

struct EnvRLayout {       // R[beta, w, beta'] without the identity channel (first)
  std::vector<int64_t> off;                // per row sector b
  std::vector<int> K;                      // columns K_b
  std::vector<std::vector<int>> col_off;   // [b][w] column offset, -1 if absent
  std::vector<std::vector<int>> b_in;      // [b][w] column sector
  int64_t size = 0;
};
EnvRLayout envR_layout(const Leg& B, const std::vector<int>& dq);

struct IsoLayout {        // U[(alpha,s),c] or V[(s,beta),c]
  std::vector<int64_t> off;                // per new sector c
  std::vector<int> rows;                   // r_c
  // row groups of sector c: (leg sector, s, row offset, dim)
  struct Grp { int sec, s, row, dim; };
  std::vector<std::vector<Grp>> grp;
  int64_t size = 0;
  int row_of(int c, int sec, int s) const;  // row offset of group or -1
};
IsoLayout U_layout(const Leg& A, const std::vector<int>& qp, const Leg& C);
IsoLayout V_layout(const Leg& B, const std::vector<int>& qp, const Leg& C);

// ---- plans

struct GemmList {
  std::vector<GemmTask> t;
  int tiles = 0;
  int tm = 64, tn = 64;              // output tile of the kernel variant
  void add(GemmTask g);              // fills tile0 / tiles_n
  double flops() const;
  void retile(int tm_, int tn_);     // recompute tile0 / tiles_n / tiles for another tile
  int tiling() const { return (tm == 128 ? 1 : 0) + (tn == 128 ? 2 : 0); }
  // fraction of MFMA work that is not padding, for tile tm_ x tn_
  double efficiency(int tm_, int tn_) const;
  void choose_tile(bool allow_large);  // picks the largest tile whose padding costs little
  // The device table of the list: the tasks, then one record whose first kXcdRanges int32 fields are the
  // per-XCD tile ranges [s_x, s_x+1) (contiguous, of about equal work: a tile costs K + 64); sets xmax, the
  // largest number of tiles of one XCD.
  std::vector<GemmTask> upload();
  int xmax = 0;
};

struct MixList {
  std::vector<MixTask> t;
  std::vector<MixSrc> src;
  int tiles = 0;
  void add(MixTask m, const std::vector<MixSrc>& s);
  double flops() const;
};

struct ScaleList {
  std::vector<ScaleTask> t;
  int tiles = 0;
  void add(ScaleTask s);
};

struct PackList {
  std::vector<PackTask> t;
  int tiles = 0;
  void add(PackTask p);              // fills RB, tile0 (256 row-chunks per tile)
};

// Words of a [R x K] matrix in the fragment layout.
int64_t frag_words(int R, int K);

struct HeffPlan {
  GemmList g1, g2;
  MixList mixY, mixT;
  std::vector<int64_t> n_psi, n_T1, n_T3;   // per problem
  std::vector<int64_t> n_L, n_R;
  // Split-bf16 policy: the same contraction on operands in the fragment layout.
  // f1/f2 are g1/g2 with aoff/boff in fragment words; mixTf is mixT writing T3
  // in the fragment layout; packL/packR (once per operator) and packX (per
  // matvec) fill the operands from the FP64 inputs.
  GemmList f1, f2;
  MixList mixYf, mixTf;
  PackList packL, packR, packX;
  std::vector<int64_t> n_Lf, n_Rf, n_Xf, n_T3f;   // words, per problem
  // The fragment form's mixing reads T1 and an FP32 copy of x (written by the x
  // pack) whose rows are padded to multiples of 4 floats and start on 16-byte
  // boundaries, so that it can read 4 columns per 16-byte load.
  std::vector<int64_t> n_T1f, n_Xm;               // floats, per problem
  // In the fragment form the K index of T3 and R (channel u, column b') is
  // re-spaced so that each channel's block starts at a multiple of 8.
  //
  // Energy shift of the low-precision copies.  Where the MPO makes L's channel
  // 0 the complete left Hamiltonian H_L (row 0 of W1 and of W2 the identity
  // alone, charge 0) and R's last channel the complete right Hamiltonian H_R
  // (last column of W2 and of W1 the identity alone, charge 0), H_eff contains
  // H_L (x) 1 and 1 (x) H_R exactly once, so the copies may hold H_L - sL and
  // H_R - sR and the result gets (sL + sR) x back in FP64.  diagL / diagR list
  // the diagonals of those blocks (the shifts are their means); shiftL / shiftR
  // say per problem whether the structure is there.
  std::vector<DiagTask> diagL, diagR;
  std::vector<int> shiftL, shiftR;
};
// heff bases: 0 L, 1 R, 2 x (GEMM operand), 3 y, 4 T1, 5 T3, 6 x (mix operand).
// Fragment form: 0 L, 1 R, 2 x, 5 T3 in the fragment layout; 3 y, 4 T1, 6 x as
// above; the packs read the FP64 L, R, x through bases 0, 1, 2 of a separate
// source table.
void build_heff(HeffPlan& p, int prob, const Leg& A, const Leg& B, const Mpo& W1, const Mpo& W2);

struct EnvPlan {
  GemmList ga, gc;
  MixList mix;
  std::vector<int64_t> n_T1, n_T2, n_new;
};
// LEFT bases: 0 L_old, 1 U, 2 L_new, 3 T_a, 4 T_2.  RIGHT bases: 0 R_old, 1 V, 2 R_new, 3 P, 4 Q.
void build_envL(EnvPlan& p, int prob, const Leg& A, const Leg& C, const Mpo& W);
void build_envR(EnvPlan& p, int prob, const Leg& B, const Leg& C, const Mpo& W);

struct PredictPlan {
  ScaleList scale;
  GemmList g;
  std::vector<int64_t> n_Vs, n_Us;
};
// bases: 0 lam_i, 1 V_i, 2 lam_prev, 3 U_ip1, 4 lam_ip1, 5 psi, 6 V scaled, 7 U scaled
void build_predict(PredictPlan& p, int prob, const Leg& Aa, const Leg& Bt, const Leg& Bb,
                   const std::vector<int>& qp);

// Charges of the fused site of two sites: qf[s1 d + s2] = qp[s1] + qp[s2].
std::vector<int> fused_qp(const std::vector<int>& qp);
// The two-site state psi (legs A, B, local charges qp) read as the right
// isometry V of the fused site with new leg A: one copy task per block of psi,
// transposed into its rows of the V layout.  bases: 0 psi, 1 V.
void build_twosite_V(MixList& m, int prob, const Leg& A, const Leg& B, const std::vector<int>& qp);
// Segments of sum_{a,a'} L[a, wl, a'] R[a, wr, a'] on one leg (L channel charges
// ql, R channel charges qr); bases 0 L, 1 R of item `item`.
void build_overlap(std::vector<OverlapSeg>& segs, int item, const Leg& leg, const std::vector<int>& ql,
                   const std::vector<int>& qr, int wl, int wr);

// Host-side bounds check of a plan before any launch: every element a task can
// touch must lie inside its base buffer.  sizes[prob * kNumBases + base] is the
// element count of that buffer (-1: unused).  Throws InvalidArg on violation.
void check_gemm(const GemmList& g, int mode, const std::vector<int64_t>& sizes, const char* what);
void check_mix(const MixList& m, const std::vector<int64_t>& sizes, const char* what);
void check_scale(const ScaleList& s, const std::vector<int64_t>& sizes, const char* what, int64_t colmap_bound);
// Fragment-layout forms (sizes of fragment buffers in 32-bit words).
void check_gemm_frag(const GemmList& g, const std::vector<int64_t>& sizes, const char* what);
void check_mix_frag(const MixList& m, const std::vector<int64_t>& sizes, const char* what);
// Sources of the 4-column mixing: non-transposed rows start at multiples of 4
// floats, have lengths that are multiples of 4, and every row's padded length
// lies inside its buffer.
void check_mix_v4(const MixList& m, const std::vector<int64_t>& sizes, const char* what);
void check_pack(const PackList& p, const std::vector<int64_t>& ssizes, const std::vector<int64_t>& dsizes,
                const char* what);

// Work of one heff_apply (flops of GEMMs and mixing; bytes of environments, x, y).
void heff_work(const Leg& A, const Leg& B, const Mpo& W1, const Mpo& W2, double& flops, double& bytes);

}  // namespace idmrg
