// Test infrastructure: executes the library's work plans on the host with
// plain loops, so that the plan builders (block bookkeeping, offsets, MPO
// mixing coefficients) can be checked against the oracle without a GPU.
// Built only by the test suite; never linked into libidmrg.so.
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
