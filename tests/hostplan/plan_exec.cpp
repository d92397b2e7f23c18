// Test infrastructure: executes the library's work plans on the host with
// plain loops, so that the plan builders (block bookkeeping, offsets, MPO
// mixing coefficients) can be checked against the oracle without a GPU.
// Built only by the test suite; never linked into libidmrg.so.
#include <cmath>
#include <cstring>
#include <vector>

#include "idmrg.h"
#include "internal.h"
#include "plan.h"

using namespace idmrg;

namespace {

double* base_ptr(const std::vector<double*>& b, int prob, int base) { return b[(size_t)prob * kNumBases + base]; }

void run_gemm(const GemmList& g, int mode, const std::vector<double*>& b) {
  for (const auto& t : g.t) {
    const double* A = base_ptr(b, t.prob, t.abase) + t.aoff;
    const double* B = base_ptr(b, t.prob, t.bbase) + t.boff;
    double* C = base_ptr(b, t.prob, t.cbase) + t.coff;
    for (int i = 0; i < t.M; ++i)
      for (int j = 0; j < t.N; ++j) {
        double s = 0.0;
        for (int k = 0; k < t.K; ++k) {
          const double a = mode == 2 ? A[(int64_t)k * t.lda + i] : A[(int64_t)i * t.lda + k];
          const double bb = mode == 1 ? B[(int64_t)j * t.ldb + k] : B[(int64_t)k * t.ldb + j];
          s += a * bb;
        }
        double& c = C[(int64_t)i * t.ldc + j];
        c = t.beta ? c + s : s;
      }
  }
}

void run_mix(const MixList& m, const std::vector<double*>& b) {
  for (const auto& t : m.t) {
    double* D = base_ptr(b, t.prob, t.dbase) + t.doff;
    for (int r = 0; r < t.rows; ++r)
      for (int c = 0; c < t.cols; ++c) {
        double s = 0.0;
        for (int k = 0; k < t.nsrc; ++k) {
          const MixSrc& x = m.src[t.src0 + k];
          const double* S = base_ptr(b, t.prob, x.base) + x.off;
          s += x.coef * (x.trans ? S[(int64_t)c * x.ld + r] : S[(int64_t)r * x.ld + c]);
        }
        D[(int64_t)r * t.ldd + c] = s;
      }
  }
}

// Fragment layout on the host: one double per bf16 slot (two per 32-bit word),
// the value in the hi slot and zero in the lo slot, so the three split-bf16
// products reduce to the exact FP64 product.
int64_t frag_slot(int64_t word_off, int KB, int r, int k) {
  return 2 * (word_off + ((int64_t)(r / kFragRows) * KB + k / kFragK) * kFragWords) + ((r % kFragRows) + 16 * ((k % kFragK) / 8)) * 8 +
         k % 8;
}

void run_pack(const PackList& pl, const std::vector<double*>& src, const std::vector<double*>& dst,
              const double* sig = nullptr) {
  for (const auto& t : pl.t) {
    const double* S = t.K > 0 ? base_ptr(src, t.prob, t.sbase) + t.soff : nullptr;
    double* D = base_ptr(dst, t.prob, t.dbase);
    for (int r = 0; r < t.RB * kFragRows; ++r)
      for (int k = 0; k < 8 * t.nch; ++k) {
        const int64_t i = frag_slot(t.doff, t.KB, r, t.kc0 + k);
        double v = r < t.R && k < t.K ? (t.trans ? S[(int64_t)k * t.ld + r] : S[(int64_t)r * t.ld + k]) : 0.0;
        if (t.xbase >= 0 && r < t.R && k < t.K) {   // the row-padded copy, in the source's orientation
          double* Xc = base_ptr(dst, t.prob, t.xbase) + t.xoff;
          if (t.trans) Xc[(int64_t)k * t.xld + r] = v;
          else Xc[(int64_t)r * t.xld + k] = v;
        }
        if (r - t.dr0 == k - t.dk0 && r - t.dr0 >= 0 && r - t.dr0 < t.dlen) v -= sig[t.shift_slot];
        D[i] = v;
        D[i + kFragWords] = 0.0;
      }
  }
}

void run_gemm_frag(const GemmList& g, const std::vector<double*>& b) {
  for (const auto& t : g.t) {
    const int KB = (t.K + kFragK - 1) / kFragK;
    const double* A = base_ptr(b, t.prob, t.abase);
    const double* B = base_ptr(b, t.prob, t.bbase);
    double* C = base_ptr(b, t.prob, t.cbase) + t.coff;
    for (int i = 0; i < t.M; ++i)
      for (int j = 0; j < t.N; ++j) {
        double s = 0.0;
        for (int k = 0; k < KB * kFragK; ++k) {   // the zero padding past K contributes nothing
          const int64_t ia = frag_slot(t.aoff, KB, i, k), ib = frag_slot(t.boff, KB, j, k);
          s += A[ia] * B[ib + kFragWords] + A[ia + kFragWords] * B[ib] + A[ia] * B[ib];
        }
        double& c = C[(int64_t)i * t.ldc + j];
        c = t.beta ? c + s : s;
      }
  }
}

void run_mix_frag(const MixList& m, const std::vector<double*>& b) {
  for (const auto& t : m.t) {
    double* D = base_ptr(b, t.prob, t.dbase);
    for (int r = 0; r < t.rows; ++r)
      for (int c = 0; c < t.cols; ++c) {
        double s = 0.0;
        for (int k = 0; k < t.nsrc; ++k) {
          const MixSrc& x = m.src[t.src0 + k];
          const double* S = base_ptr(b, t.prob, x.base) + x.off;
          s += x.coef * (x.trans ? S[(int64_t)c * x.ld + r] : S[(int64_t)r * x.ld + c]);
        }
        const int64_t i = frag_slot(t.doff, t.ldd, t.r0 + r, t.c0 + c);
        D[i] = s;
        D[i + kFragWords] = 0.0;
      }
    // the chunk holding the last column is written whole: zeros past it
    for (int r = 0; r < t.rows; ++r)
      for (int c = t.cols; c % 8 != 0; ++c) {
        const int64_t i = frag_slot(t.doff, t.ldd, t.r0 + r, t.c0 + c);
        D[i] = 0.0;
        D[i + kFragWords] = 0.0;
      }
  }
}

}  // namespace

extern "C" int hostplan_heff(const idmrg_heff* H, const double* x, double* y) {
  try {
    HeffPlan p;
    const Leg A = make_leg(H->left, "A"), B = make_leg(H->right, "B");
    build_heff(p, 0, A, B, make_mpo(H->w1, "w1"), make_mpo(H->w2, "w2"));
    std::vector<double> T1(p.n_T1[0] + 1), T3(p.n_T3[0] + 1);
    std::vector<double*> b(kNumBases, nullptr);
    b[0] = (double*)H->L; b[1] = (double*)H->R; b[2] = (double*)x; b[3] = y; b[4] = T1.data(); b[5] = T3.data();
    b[6] = (double*)x;
    std::vector<int64_t> sz(kNumBases, -1);
    sz[0] = p.n_L[0]; sz[1] = p.n_R[0]; sz[2] = sz[3] = sz[6] = p.n_psi[0]; sz[4] = p.n_T1[0]; sz[5] = p.n_T3[0];
    check_gemm(p.g1, 0, sz, "g1");
    check_mix(p.mixY, sz, "mixY");
    check_mix(p.mixT, sz, "mixT");
    check_gemm(p.g2, 1, sz, "g2");
    run_gemm(p.g1, 0, b);
    run_mix(p.mixY, b);
    run_mix(p.mixT, b);
    run_gemm(p.g2, 1, b);
    return 0;
  } catch (...) {
    return -1;
  }
}

// The split-bf16 form of the same plan: packs, fragment GEMMs and the mixing
// into the fragment form of T3.  Fragment buffers start as NaN except T3's,
// which starts as zero like its device buffer, so a read of any slot that no
// pack wrote shows up in y.  The packs shift the H_L and H_R diagonals by sL
// and sR where the plan found that structure (flags[0], flags[1] on return),
// and (sL + sR) x is added back, as on the device.
extern "C" int hostplan_heff_frag(const idmrg_heff* H, const double* x, double* y, double sL, double sR,
                                  int* flags) {
  try {
    HeffPlan p;
    const Leg A = make_leg(H->left, "A"), B = make_leg(H->right, "B");
    build_heff(p, 0, A, B, make_mpo(H->w1, "w1"), make_mpo(H->w2, "w2"));
    const double nan = std::nan("");
    std::vector<double> Lf(2 * p.n_Lf[0] + 2, nan), Rf(2 * p.n_Rf[0] + 2, nan), Xf(2 * p.n_Xf[0] + 2, nan),
        T1(p.n_T1f[0] + 1, nan), Xm(p.n_Xm[0] + 1, nan), T3f(2 * p.n_T3f[0] + 2, 0.0);
    std::vector<double*> src(kNumBases, nullptr), b(kNumBases, nullptr);
    src[0] = (double*)H->L; src[1] = (double*)H->R; src[2] = (double*)x;
    b[0] = Lf.data(); b[1] = Rf.data(); b[2] = Xf.data(); b[3] = y; b[4] = T1.data(); b[5] = T3f.data();
    b[6] = Xm.data();
    std::vector<int64_t> ss(kNumBases, -1), sz(kNumBases, -1);
    ss[0] = p.n_L[0]; ss[1] = p.n_R[0]; ss[2] = p.n_psi[0];
    sz[0] = p.n_Lf[0]; sz[1] = p.n_Rf[0]; sz[2] = p.n_Xf[0]; sz[3] = p.n_psi[0]; sz[4] = p.n_T1f[0];
    sz[5] = p.n_T3f[0]; sz[6] = p.n_Xm[0];
    flags[0] = p.shiftL[0];
    flags[1] = p.shiftR[0];
    const double sig[2] = {p.shiftL[0] ? sL : 0.0, p.shiftR[0] ? sR : 0.0};   // slots 0 (left), 1 (right)
    const double sigma = sig[0] + sig[1];
    check_pack(p.packL, ss, sz, "packL");
    check_pack(p.packR, ss, sz, "packR");
    check_pack(p.packX, ss, sz, "packX");
    check_gemm_frag(p.f1, sz, "f1");
    check_mix(p.mixYf, sz, "mixYf");
    check_mix_v4(p.mixYf, sz, "mixYf");
    check_mix_frag(p.mixTf, sz, "mixTf");
    check_mix_v4(p.mixTf, sz, "mixTf");
    check_gemm_frag(p.f2, sz, "f2");
    run_pack(p.packL, src, b, sig);
    run_pack(p.packR, src, b, sig);
    run_pack(p.packX, src, b, sig);
    run_gemm_frag(p.f1, b);
    run_mix(p.mixYf, b);
    run_mix_frag(p.mixTf, b);
    run_gemm_frag(p.f2, b);
    for (int64_t i = 0; i < p.n_psi[0]; ++i) y[i] += sigma * x[i];
    return 0;
  } catch (...) {
    return -1;
  }
}

extern "C" int hostplan_env(int side, const idmrg_env_update* u) {
  try {
    EnvPlan p;
    const Leg O = make_leg(u->old_leg, "old"), C = make_leg(u->new_leg, "new");
    const Mpo W = make_mpo(u->w, "w");
    if (side == IDMRG_LEFT) build_envL(p, 0, O, C, W);
    else build_envR(p, 0, O, C, W);
    std::vector<double> T1(p.n_T1[0] + 1), T2(p.n_T2[0] + 1);
    std::vector<double*> b(kNumBases, nullptr);
    b[0] = (double*)u->env_old; b[1] = (double*)u->iso; b[2] = u->env_new; b[3] = T1.data(); b[4] = T2.data();
    std::vector<int64_t> sz(kNumBases, -1);
    if (side == IDMRG_LEFT) {
      sz[0] = envL_layout(O, W.ql).size; sz[1] = U_layout(O, W.qp, C).size; sz[2] = envL_layout(C, W.qr).size;
    } else {
      sz[0] = envR_layout(O, W.qr).size; sz[1] = V_layout(O, W.qp, C).size; sz[2] = envR_layout(C, W.ql).size;
    }
    sz[3] = p.n_T1[0]; sz[4] = p.n_T2[0];
    check_gemm(p.ga, side == IDMRG_LEFT ? 0 : 2, sz, "ga");
    check_mix(p.mix, sz, "mix");
    check_gemm(p.gc, side == IDMRG_LEFT ? 2 : 0, sz, "gc");
    run_gemm(p.ga, side == IDMRG_LEFT ? 0 : 2, b);
    run_mix(p.mix, b);
    run_gemm(p.gc, side == IDMRG_LEFT ? 2 : 0, b);
    return 0;
  } catch (...) {
    return -1;
  }
}

// A two-site state as the right isometry of its fused site (twosite_to_right_iso's plan).
extern "C" int hostplan_twosite_V(const idmrg_leg* left, const idmrg_leg* right, int d, const int32_t* qp_in,
                                  const double* psi, double* out) {
  try {
    const Leg A = make_leg(*left, "A"), B = make_leg(*right, "B");
    const std::vector<int> qp = make_qp(d, qp_in);
    MixList m;
    build_twosite_V(m, 0, A, B, qp);
    std::vector<int64_t> sz(kNumBases, -1);
    sz[0] = psi_layout(A, B, qp).size;
    sz[1] = V_layout(B, fused_qp(qp), A).size;
    check_mix(m, sz, "twosite");
    std::vector<double*> b(kNumBases, nullptr);
    b[0] = (double*)psi;
    b[1] = out;
    run_mix(m, b);
    return 0;
  } catch (...) {
    return -1;
  }
}

// env_overlap's segments, summed with plain loops.
extern "C" int hostplan_overlap(const idmrg_overlap_item* it, double* out) {
  try {
    const Leg leg = make_leg(it->leg, "leg");
    const std::vector<int> ql(it->ql, it->ql + it->nl), qr(it->qr, it->qr + it->nr);
    std::vector<OverlapSeg> segs;
    build_overlap(segs, 0, leg, ql, qr, it->wl, it->wr);
    double s = 0.0;
    for (const OverlapSeg& g : segs)
      for (int i = 0; i < g.rows; ++i)
        for (int j = 0; j < g.cols; ++j) s += it->L[g.aoff + (int64_t)i * g.lda + j] * it->R[g.boff + (int64_t)i * g.ldb + j];
    *out = s;
    return 0;
  } catch (...) {
    return -1;
  }
}

// The per-XCD tile ranges stored after a GEMM task table (stage 1 and 2 of the split-bf16 plan, 128 x 128 tiles):
// out[0..8] the ranges, out[9] the largest range, out[10] the tile count, out[11..18] each XCD's work (K + 64 per
// tile) in units of the largest single tile's work.
extern "C" int hostplan_xcd_ranges(const idmrg_heff* H, int nprob, int stage, double* out) {
  try {
    HeffPlan p;
    for (int i = 0; i < nprob; ++i)
      build_heff(p, i, make_leg(H[i].left, "A"), make_leg(H[i].right, "B"), make_mpo(H[i].w1, "w1"),
                 make_mpo(H[i].w2, "w2"));
    GemmList g = stage == 1 ? p.f1 : p.f2;
    g.retile(128, 128);
    const std::vector<GemmTask> up = g.upload();
    if (up.size() != g.t.size() + 1) return -2;
    int32_t s[kXcdRanges];
    std::memcpy(s, &up.back(), sizeof(s));
    for (int i = 0; i < kXcdRanges; ++i) out[i] = s[i];
    out[kXcdRanges] = g.xmax;
    out[kXcdRanges + 1] = g.tiles;
    double big = 0.0;
    std::vector<double> cost(g.tiles, 0.0);
    for (size_t k = 0; k + 1 < up.size(); ++k) {   // the uploaded order, whose tile0 the ranges refer to
      const GemmTask& t = up[k];
      if (k > 0 && t.tile0 < up[k - 1].tile0) return -3;
      const int nt = ((t.M + 127) / 128) * t.tiles_n;
      for (int i = 0; i < nt; ++i) cost[t.tile0 + i] = std::max(t.K, 0) + 64;
      big = std::max(big, (double)std::max(t.K, 0) + 64);
    }
    for (int x = 0; x + 1 < kXcdRanges; ++x) {
      double w = 0.0;
      for (int i = s[x]; i < s[x + 1]; ++i) w += cost[i];
      out[kXcdRanges + 2 + x] = w / big;
    }
    return 0;
  } catch (...) {
    return -1;
  }
}
