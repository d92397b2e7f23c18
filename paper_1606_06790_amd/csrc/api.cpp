// C-ABI entry points (idmrg.h): validation, workspace, plan upload and the
// launch sequences of the five calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>

#include "idmrg.h"
#include "internal.h"
#include "plan.h"

using namespace idmrg;

// ------------------------------------------------------------------ context

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t n = 0;
};

}  // namespace

namespace {
struct ProfRec {
  int cls;
  hipEvent_t a, b;
  double flops;
};
}  // namespace

struct idmrg_ctx {
  int device = 0;
  // profiling (see idmrg_profile)
  bool prof = false;
  std::vector<ProfRec> pending;
  std::vector<hipEvent_t> pool;
  int64_t prof_n[IDMRG_PROF_CLASSES] = {};
  double prof_ms[IDMRG_PROF_CLASSES] = {};
  double prof_flops[IDMRG_PROF_CLASSES] = {};
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;   // graph capture only (nothing executes on it); created on first use
  std::string err;
  DevBuf plan;                 // uploaded task lists and base tables
  void* pinned = nullptr;      // host staging for uploads
  size_t pinned_n = 0;
  DevBuf ws[20];               // scratch, by purpose (see WS_*)
  // GEMM tile autotuner: measured best tiling per (precision, stage, shape bucket)
  std::map<std::tuple<int, int, int, int, int>, int> tune;
  hipEvent_t tev[4][4] = {};   // [variant][stage-1 start, stage-1 end, stage-2 start, stage-2 end]
};

namespace {

enum {
  WS_T1 = 0, WS_T3, WS_LOWENV, WS_LOWVEC, WS_LZ, WS_LZSMALL, WS_SVD, WS_SEL, WS_ENV, WS_PRED, WS_READ, WS_MISC,
  WS_PLAN64, WS_PLANLOW, WS_T3F, WS_DIAG, WS_BJ, WS_T1LO
};

void sync(idmrg_ctx* c) { IDMRG_HIP(hipStreamSynchronize(c->stream)); }

hipEvent_t take_event(idmrg_ctx* c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e;
  IDMRG_HIP(hipEventCreate(&e));
  return e;
}

// Brackets the launches issued during its lifetime with events (if profiling).
struct Prof {
  idmrg_ctx* c;
  ProfRec r{};
  Prof(idmrg_ctx* ctx, int cls, double flops) : c(ctx) {
    if (!c->prof) return;
    r.cls = cls;
    r.flops = flops;
    r.a = take_event(c);
    r.b = take_event(c);
    IDMRG_HIP(hipEventRecord(r.a, c->stream));
  }
  ~Prof() {
    if (!c->prof) return;
    if (hipEventRecord(r.b, c->stream) == hipSuccess) c->pending.push_back(r);
  }
};

void prof_collect(idmrg_ctx* c) {
  if (c->pending.empty()) return;
  IDMRG_HIP(hipStreamSynchronize(c->stream));
  for (auto& r : c->pending) {
    float ms = 0.f;
    IDMRG_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    c->prof_n[r.cls] += 1;
    c->prof_ms[r.cls] += ms;
    c->prof_flops[r.cls] += r.flops;
    c->pool.push_back(r.a);
    c->pool.push_back(r.b);
  }
  c->pending.clear();
}

void* ensure(idmrg_ctx* c, DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (b.n >= bytes) return b.p;
  sync(c);
  size_t want = std::max(bytes, b.n + b.n / 4);
  if (b.p) IDMRG_HIP(hipFree(b.p));
  b.p = nullptr;
  b.n = 0;
  want = (want + 4095) / 4096 * 4096;
  if (hipMalloc(&b.p, want) != hipSuccess) {
    b.p = nullptr;
    (void)hipGetLastError();
    throw std::bad_alloc();
  }
  b.n = want;
  return b.p;
}

// Collects host arrays into one upload; offsets aligned to 256 bytes.
struct Packer {
  std::vector<char> host;
  size_t add(const void* p, size_t bytes) {
    const size_t off = (host.size() + 255) / 256 * 256;
    host.resize(off + std::max<size_t>(bytes, 8));
    if (bytes) std::memcpy(host.data() + off, p, bytes);
    return off;
  }
  template <typename T>
  size_t add(const std::vector<T>& v) { return add(v.data(), v.size() * sizeof(T)); }
};

char* upload(idmrg_ctx* c, const Packer& pk, DevBuf* target = nullptr) {
  sync(c);   // previous work may still read the plan buffer and the staging area
  char* dev = (char*)ensure(c, target ? *target : c->plan, pk.host.size());
  if (c->pinned_n < pk.host.size()) {
    if (c->pinned) IDMRG_HIP(hipHostFree(c->pinned));
    c->pinned = nullptr;
    c->pinned_n = 0;
    size_t want = std::max(pk.host.size(), (size_t)1 << 20);
    IDMRG_HIP(hipHostMalloc(&c->pinned, want, hipHostMallocDefault));
    c->pinned_n = want;
  }
  std::memcpy(c->pinned, pk.host.data(), pk.host.size());
  IDMRG_HIP(hipMemcpyAsync(dev, c->pinned, pk.host.size(), hipMemcpyHostToDevice, c->stream));
  return dev;
}

template <typename F>
int guarded(idmrg_ctx* c, F&& f) {
  if (!c) return IDMRG_EINVAL;
  try {
    c->err.clear();
    IDMRG_HIP(hipSetDevice(c->device));
    return f();
  } catch (const InvalidArg& e) {
    c->err = e.what;
    return IDMRG_EINVAL;
  } catch (const HipFailure& e) {
    c->err = e.what;
    return IDMRG_EHIP;
  } catch (const std::bad_alloc&) {
    c->err = "device or host allocation failed";
    return IDMRG_ENOMEM;
  } catch (...) {
    c->err = "unexpected internal error";
    return IDMRG_EUNSUPPORTED;
  }
}

// The caller's buffer at p must hold n elements of esize bytes inside one device allocation.
void check_dev(const void* p, int64_t n, size_t esize, const std::string& what) {
  if (!p) throw InvalidArg(what + ": null pointer");
  if (n <= 0) return;
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p) != hipSuccess) {
    (void)hipGetLastError();
    throw InvalidArg(what + ": not a device allocation of this context's device");
  }
  if ((const char*)p + (size_t)n * esize > (const char*)base + size) throw InvalidArg(what + ": buffer too small");
}

// ------------------------------------------------------------------ H_eff execution

// Output tilings of the FP64/FP32 GEMM kernel: code c -> (c & 1 ? 128 : 64) x (c & 2 ? 128 : 64).
constexpr int kTilings = 4;

struct HeffExec {
  HeffPlan plan;
  int P = 0;
  Prec prec = Prec::F64;
  // every tiling variant of both GEMM stages is uploaded; sel[stage] is the one in use
  GemmTask* gv[2][kTilings] = {};
  int tiles[2][kTilings] = {};
  int code[kTilings] = {};
  int nvar = 1;
  int sel[2] = {0, 0};
  bool need_tune[2] = {false, false};
  std::tuple<int, int, int, int, int> key[2];
  MixTask *mY = nullptr, *mT = nullptr;
  MixSrc *sY = nullptr, *sT = nullptr;
  void** bases = nullptr;      // device [P][8]
  // split-bf16: FP64 sources of the fragment packs (device [P][8]: 0 L, 1 R, 2 x) and the per-matvec x pack
  void** sbases = nullptr;
  PackTask* pX = nullptr;
  // per-problem buffers of the low-precision policies (xlow: the GEMM operand, xmix: FP32 x for the mixing)
  std::vector<void*> xlow, xmix, ylow;
  std::vector<int64_t> npsi;
  // energy shift of the low-precision copies: y = (H - sigma) x in low precision + sigma x in FP64
  std::vector<double> sigma;
  double flops_g1 = 0, flops_g2 = 0, flops_mix = 0;
};

size_t elem_size_operand(Prec p) { return p == Prec::F64 ? 8 : 4; }

int ilog2(double x) { return x >= 1.0 ? (int)std::floor(std::log2(x)) : 0; }

// Shape bucket of one GEMM stage: precision, stage, log2 of the flops and of
// the flop-weighted mean N and K (the tile choice depends on these, not on
// the exact block dimensions, which change a little every iteration).
std::tuple<int, int, int, int, int> tune_key(Prec prec, int stage, const GemmList& g) {
  double f = 0, fn = 0, fk = 0;
  for (const auto& t : g.t) {
    const double w = 2.0 * t.M * (double)t.N * t.K;
    f += w;
    fn += w * t.N;
    fk += w * t.K;
  }
  return std::make_tuple((int)prec, stage, ilog2(f), f > 0 ? ilog2(fn / f) : 0, f > 0 ? ilog2(fk / f) : 0);
}

// After the trial matvecs of every variant have completed: keep the fastest
// tiling of each stage that still needed tuning, and remember it.
void tune_resolve(idmrg_ctx* c, HeffExec& ex, int ntried) {
  if (ntried < 1) return;
  for (int st = 0; st < 2; ++st) {
    if (!ex.need_tune[st]) continue;
    int best = -1;
    float bms = 0.f;
    for (int v = 0; v < ntried; ++v) {
      float ms = 0.f;
      IDMRG_HIP(hipEventElapsedTime(&ms, c->tev[v][2 * st], c->tev[v][2 * st + 1]));
      if (best < 0 || ms < bms) best = v, bms = ms;
    }
    ex.sel[st] = best;
    ex.need_tune[st] = false;
    if (ntried == ex.nvar) c->tune[ex.key[st]] = best;
  }
}

// Build plans for P problems, allocate scratch, convert environments for the
// low-precision policies, and upload.  x/y are the FP64 input/output vectors.
void heff_setup(idmrg_ctx* c, HeffExec& ex, int P, const idmrg_heff* H, const std::vector<double*>& x,
                const std::vector<double*>& y, int prec, DevBuf* planbuf = nullptr) {
  if (prec < 0 || prec > 2) throw InvalidArg("unknown precision policy");
  ex.P = P;
  ex.prec = (Prec)prec;
  std::vector<Leg> A(P), B(P);
  std::vector<Mpo> W1(P), W2(P);
  for (int p = 0; p < P; ++p) {
    if (!H[p].w1 || !H[p].w2 || !H[p].L || !H[p].R) throw InvalidArg("null field in idmrg_heff");
    A[p] = make_leg(H[p].left, "heff.left");
    B[p] = make_leg(H[p].right, "heff.right");
    W1[p] = make_mpo(H[p].w1, "heff.w1");
    W2[p] = make_mpo(H[p].w2, "heff.w2");
    if (W1[p].dr != W2[p].dl || W1[p].qr != W2[p].ql) throw InvalidArg("w1 columns and w2 rows differ");
    if (W1[p].qp != W2[p].qp) throw InvalidArg("w1 and w2 local charges differ");
    build_heff(ex.plan, p, A[p], B[p], W1[p], W2[p]);
    if (ex.plan.n_psi[p] == 0) throw InvalidArg("two-site state has no allowed block");
  }
  ex.npsi = ex.plan.n_psi;
  const bool frag = ex.prec == Prec::BF16X3;
  // Tile variants.  The tile shape does not change the order in which any
  // output element accumulates over k, so all variants give identical results.
  std::vector<GemmList> var[2];
  ex.nvar = kTilings;
  for (int v = 0; v < kTilings; ++v) ex.code[v] = v;
  for (int st = 0; st < 2; ++st) {
    const GemmList& base = st == 0 ? (frag ? ex.plan.f1 : ex.plan.g1) : (frag ? ex.plan.f2 : ex.plan.g2);
    for (int v = 0; v < ex.nvar; ++v) {
      var[st].push_back(base);
      var[st][v].retile(ex.code[v] & 1 ? 128 : 64, ex.code[v] & 2 ? 128 : 64);
      ex.tiles[st][v] = var[st][v].tiles;
    }
    ex.key[st] = tune_key(ex.prec, st, base);
    auto it = c->tune.find(ex.key[st]);
    ex.need_tune[st] = ex.nvar > 1 && it == c->tune.end();
    if (it != c->tune.end()) {
      ex.sel[st] = it->second;
    } else {   // untuned default: padding heuristic, except 64 x 64 for FP64 (its larger tiles run one wave per SIMD)
      GemmList h = base;
      h.choose_tile(ex.prec != Prec::F64);
      ex.sel[st] = h.tiling();
    }
  }
  ex.flops_g1 = ex.plan.g1.flops();
  ex.flops_g2 = ex.plan.g2.flops();
  ex.flops_mix = ex.plan.mixY.flops() + ex.plan.mixT.flops();
  {
    std::vector<int64_t> sz((size_t)P * kNumBases, -1);
    for (int p = 0; p < P; ++p) {
      int64_t* z = &sz[(size_t)p * kNumBases];
      z[0] = ex.plan.n_L[p]; z[1] = ex.plan.n_R[p]; z[2] = z[3] = z[6] = ex.plan.n_psi[p];
      z[4] = ex.plan.n_T1[p]; z[5] = ex.plan.n_T3[p];
      check_dev(H[p].L, ex.plan.n_L[p], 8, "heff.L");
      check_dev(H[p].R, ex.plan.n_R[p], 8, "heff.R");
      check_dev(x[p], ex.plan.n_psi[p], 8, "x");
      check_dev(y[p], ex.plan.n_psi[p], 8, "y");
    }
    if (!frag) {
      check_gemm(ex.plan.g1, 0, sz, "heff gemm1");
      check_mix(ex.plan.mixY, sz, "heff mixY");
      check_mix(ex.plan.mixT, sz, "heff mixT");
      check_gemm(ex.plan.g2, 1, sz, "heff gemm2");
    } else {
      std::vector<int64_t> ss = sz;   // FP64 sources of the packs: 0 L, 1 R, 2 x
      for (int p = 0; p < P; ++p) {
        int64_t* z = &sz[(size_t)p * kNumBases];
        z[0] = ex.plan.n_Lf[p]; z[1] = ex.plan.n_Rf[p]; z[2] = ex.plan.n_Xf[p]; z[5] = ex.plan.n_T3f[p];
        z[4] = ex.plan.n_T1f[p]; z[6] = ex.plan.n_Xm[p];
      }
      check_gemm_frag(ex.plan.f1, sz, "heff gemm1");
      check_mix(ex.plan.mixYf, sz, "heff mixY");
      check_mix_v4(ex.plan.mixYf, sz, "heff mixY");
      check_mix_frag(ex.plan.mixTf, sz, "heff mixT");
      check_mix_v4(ex.plan.mixTf, sz, "heff mixT");
      check_gemm_frag(ex.plan.f2, sz, "heff gemm2");
      check_pack(ex.plan.packL, ss, sz, "heff pack L");
      check_pack(ex.plan.packR, ss, sz, "heff pack R");
      check_pack(ex.plan.packX, ss, sz, "heff pack x");
    }
  }
  const size_t es = ex.prec == Prec::F64 ? 8 : 4;   // accumulator / T1 element size
  // sub-buffers start at multiples of 64 elements (256 bytes), which the 16-byte accesses of the split-bf16 kernels need
  auto round64 = [](int64_t n) { return (n + 63) / 64 * 64; };
  int64_t nT1 = 0, nT3 = 0;
  std::vector<int64_t> o1(P), o3(P);
  for (int p = 0; p < P; ++p) {
    o1[p] = nT1;
    o3[p] = nT3;
    nT1 += round64((frag ? ex.plan.n_T1f[p] : ex.plan.n_T1[p]) + 1);
    nT3 += round64((frag ? ex.plan.n_T3f[p] : ex.plan.n_T3[p]) + 1);
  }
  // the FP64 and the low-precision plans of one Lanczos call are live together, so each has its own T1 and T3
  char* T1 = (char*)ensure(c, c->ws[ex.prec == Prec::F64 ? WS_T1 : WS_T1LO], nT1 * es);
  char* T3 = (char*)ensure(c, c->ws[ex.prec == Prec::F64 ? WS_T3 : WS_T3F], nT3 * es);
  // the fragment form of T3 is written only inside its blocks: its padding stays zero from here on
  if (frag) IDMRG_HIP(hipMemsetAsync(T3, 0, nT3 * es, c->stream));
  std::vector<void*> hb((size_t)P * kNumBases, nullptr), sb;
  ex.xlow.assign(P, nullptr);
  ex.xmix.assign(P, nullptr);
  ex.ylow.assign(P, nullptr);
  if (ex.prec == Prec::F64) {
    for (int p = 0; p < P; ++p) {
      void** b = &hb[(size_t)p * kNumBases];
      b[0] = (void*)H[p].L;
      b[1] = (void*)H[p].R;
      b[2] = x[p];
      b[3] = y[p];
      b[4] = T1 + o1[p] * 8;
      b[5] = T3 + o3[p] * 8;
      b[6] = x[p];
    }
  } else {
    // 4-byte units: FP32 L, R, x (also the mixing operand), y; or, for split-bf16,
    // fragment-layout L, R, x, plus FP32 x for the mixing and y
    const std::vector<int64_t>& nL = frag ? ex.plan.n_Lf : ex.plan.n_L;
    const std::vector<int64_t>& nR = frag ? ex.plan.n_Rf : ex.plan.n_R;
    int64_t nenv = 0, nvec = 0;
    for (int p = 0; p < P; ++p) {
      nenv += round64(nL[p]) + round64(nR[p]);
      nvec += (frag ? round64(ex.plan.n_Xf[p]) + round64(ex.plan.n_Xm[p]) : round64(ex.npsi[p])) + round64(ex.npsi[p]);
    }
    char* env = (char*)ensure(c, c->ws[WS_LOWENV], nenv * 4);
    char* vec = (char*)ensure(c, c->ws[WS_LOWVEC], nvec * 4);
    int64_t oe = 0, ov = 0;
    if (frag) sb.assign((size_t)P * kNumBases, nullptr);
    for (int p = 0; p < P; ++p) {
      void** b = &hb[(size_t)p * kNumBases];
      void* Ll = env + oe * 4;
      oe += round64(nL[p]);
      void* Rl = env + oe * 4;
      oe += round64(nR[p]);
      ex.xmix[p] = vec + ov * 4;   // split-bf16: the row-padded copy the x pack writes
      ov += round64(frag ? ex.plan.n_Xm[p] : ex.npsi[p]);
      ex.ylow[p] = vec + ov * 4;
      ov += round64(ex.npsi[p]);
      if (frag) {
        ex.xlow[p] = vec + ov * 4;
        ov += round64(ex.plan.n_Xf[p]);
        void** q = &sb[(size_t)p * kNumBases];
        q[0] = (void*)H[p].L;
        q[1] = (void*)H[p].R;
        q[2] = x[p];
      } else {
        ex.xlow[p] = ex.xmix[p];
        launch_convert(0, H[p].L, Ll, ex.plan.n_L[p], c->stream);
        launch_convert(0, H[p].R, Rl, ex.plan.n_R[p], c->stream);
      }
      b[0] = Ll;
      b[1] = Rl;
      b[2] = ex.xlow[p];
      b[3] = ex.ylow[p];
      b[4] = T1 + o1[p] * 4;
      b[5] = T3 + o3[p] * 4;
      b[6] = ex.xmix[p];
    }
  }
  // Energy shift of the low-precision copies (see plan.h): sL, sR = mean
  // diagonal of the H_L and H_R blocks, from their FP64 sources.
  ex.sigma.assign(P, 0.0);
  std::vector<DiagTask> diag = ex.plan.diagL;
  diag.insert(diag.end(), ex.plan.diagR.begin(), ex.plan.diagR.end());
  const size_t nDL = ex.plan.diagL.size();
  std::vector<double> dshift(diag.size(), 0.0);
  char* dd = nullptr;
  size_t d1 = 0, d3 = 0;
  if (ex.prec != Prec::F64 && !diag.empty()) {
    if (sb.empty()) {
      sb.assign((size_t)P * kNumBases, nullptr);
      for (int p = 0; p < P; ++p) {
        sb[(size_t)p * kNumBases + 0] = (void*)H[p].L;
        sb[(size_t)p * kNumBases + 1] = (void*)H[p].R;
        sb[(size_t)p * kNumBases + 2] = x[p];
      }
    }
    Packer dk;
    d1 = dk.add(diag);
    const size_t d2 = dk.add(sb);
    d3 = dk.add(dshift);
    dd = upload(c, dk, &c->ws[WS_DIAG]);
    launch_diag_sum((const DiagTask*)(dd + d1), (int)diag.size(), (void* const*)(dd + d2), (double*)(dd + d3),
                    c->stream);
    std::vector<double> sums(diag.size());
    IDMRG_HIP(hipMemcpyAsync(sums.data(), dd + d3, sums.size() * 8, hipMemcpyDeviceToHost, c->stream));
    sync(c);
    std::vector<double> sL(P, 0.0), sR(P, 0.0), nL(P, 0.0), nR(P, 0.0);
    for (size_t t = 0; t < diag.size(); ++t) {
      const int p = diag[t].prob;
      (t < nDL ? sL : sR)[p] += sums[t];
      (t < nDL ? nL : nR)[p] += diag[t].len;
    }
    for (int p = 0; p < P; ++p) {
      sL[p] = (ex.plan.shiftL[p] && nL[p] > 0) ? sL[p] / nL[p] : 0.0;
      sR[p] = (ex.plan.shiftR[p] && nR[p] > 0) ? sR[p] / nR[p] : 0.0;
      ex.sigma[p] = sL[p] + sR[p];
    }
    for (auto& t : ex.plan.packL.t) t.shift = t.dlen > 0 ? sL[t.prob] : 0.0;
    for (auto& t : ex.plan.packR.t) t.shift = t.dlen > 0 ? sR[t.prob] : 0.0;
    for (size_t t = 0; t < diag.size(); ++t) dshift[t] = (t < nDL ? sL : sR)[diag[t].prob];
    IDMRG_HIP(hipMemcpyAsync(dd + d3, dshift.data(), dshift.size() * 8, hipMemcpyHostToDevice, c->stream));
    sync(c);   // dshift is a host vector
  }
  Packer pk;
  size_t av[2][kTilings];
  for (int st = 0; st < 2; ++st)
    for (int v = 0; v < ex.nvar; ++v) av[st][v] = pk.add(var[st][v].t);
  const MixList& mY = frag ? ex.plan.mixYf : ex.plan.mixY;
  const MixList& mT = frag ? ex.plan.mixTf : ex.plan.mixT;
  const size_t a3 = pk.add(mY.t), a4 = pk.add(mY.src), a5 = pk.add(mT.t), a6 = pk.add(mT.src), a7 = pk.add(hb);
  size_t a8 = 0, a9 = 0, a10 = 0, a11 = 0;
  if (!sb.empty()) a8 = pk.add(sb);
  if (frag) {
    a9 = pk.add(ex.plan.packX.t);
    a10 = pk.add(ex.plan.packL.t);
    a11 = pk.add(ex.plan.packR.t);
  }
  char* dev = upload(c, pk, planbuf);
  for (int st = 0; st < 2; ++st)
    for (int v = 0; v < ex.nvar; ++v) ex.gv[st][v] = (GemmTask*)(dev + av[st][v]);
  ex.mY = (MixTask*)(dev + a3);
  ex.sY = (MixSrc*)(dev + a4);
  ex.mT = (MixTask*)(dev + a5);
  ex.sT = (MixSrc*)(dev + a6);
  ex.bases = (void**)(dev + a7);
  if (!sb.empty()) ex.sbases = (void**)(dev + a8);
  if (ex.prec == Prec::F32 && dd)   // the FP32 copies of the H_L, H_R diagonals, shifted, from the FP64 sources
    launch_diag_shift_f32((const DiagTask*)(dd + d1), (int)diag.size(), ex.sbases, ex.bases,
                          (const double*)(dd + d3), c->stream);
  if (frag) {
    // operands fixed for the whole operator: packed once here
    ex.pX = (PackTask*)(dev + a9);
    launch_pack((PackTask*)(dev + a10), (int)ex.plan.packL.t.size(), ex.plan.packL.tiles, ex.sbases, ex.bases, nullptr,
                c->stream);
    launch_pack((PackTask*)(dev + a11), (int)ex.plan.packR.t.size(), ex.plan.packR.tiles, ex.sbases, ex.bases, nullptr,
                c->stream);
    IDMRG_HIP(hipGetLastError());
  }
}

// y = H x for every problem (x, y: the FP64 vectors given at setup).
// trial >= 0: run tiling variant `trial` in both stages and bracket each stage with the tuning events.
void heff_run(idmrg_ctx* c, HeffExec& ex, const std::vector<double*>& x, const std::vector<double*>& y,
              const int32_t* active, int trial = -1) {
  hipStream_t s = c->stream;
  if (ex.prec != Prec::F64) {
    Prof pr(c, 3, 0.0);
    if (ex.prec == Prec::BF16X3)   // also writes the padded FP32 copy of x for the mixing
      launch_pack(ex.pX, (int)ex.plan.packX.t.size(), ex.plan.packX.tiles, ex.sbases, ex.bases, active, s);
    else
      for (int p = 0; p < ex.P; ++p) launch_convert(0, x[p], ex.xmix[p], ex.npsi[p], s);
  }
  const bool frag = ex.prec == Prec::BF16X3;
  const int tin = ex.prec == Prec::F64 ? 0 : (frag ? 4 : 1);
  const int toutT = ex.prec == Prec::F64 ? 0 : (ex.prec == Prec::F32 ? 1 : 3);
  const int toutY = ex.prec == Prec::F64 ? 0 : 1;
  const int lo = ex.prec == Prec::F64 ? 0 : 9;   // profile classes of the low-precision policies
  const int v1 = trial >= 0 ? trial : ex.sel[0], v2 = trial >= 0 ? trial : ex.sel[1];
  {
    Prof pr(c, lo + 0, ex.flops_g1);
    if (trial >= 0) IDMRG_HIP(hipEventRecord(c->tev[trial][0], s));
    launch_gemm(ex.prec, 0, ex.gv[0][v1], (int)ex.plan.g1.t.size(), ex.tiles[0][v1], ex.bases, active, s,
                ex.code[v1]);
    if (trial >= 0) IDMRG_HIP(hipEventRecord(c->tev[trial][1], s));
  }
  {
    Prof pr(c, lo + 2, ex.flops_mix);
    const MixList& mY = frag ? ex.plan.mixYf : ex.plan.mixY;
    launch_mix(tin, toutY, ex.mY, ex.sY, (int)mY.t.size(), mY.tiles, ex.bases, active, s);
    const MixList& mT = frag ? ex.plan.mixTf : ex.plan.mixT;
    launch_mix(tin, toutT, ex.mT, ex.sT, (int)mT.t.size(), mT.tiles, ex.bases, active, s);
  }
  {
    Prof pr(c, lo + 1, ex.flops_g2);
    if (trial >= 0) IDMRG_HIP(hipEventRecord(c->tev[trial][2], s));
    launch_gemm(ex.prec, 1, ex.gv[1][v2], (int)ex.plan.g2.t.size(), ex.tiles[1][v2], ex.bases, active, s,
                ex.code[v2]);
    if (trial >= 0) IDMRG_HIP(hipEventRecord(c->tev[trial][3], s));
  }
  if (ex.prec != Prec::F64) {
    Prof pr(c, 3, 0.0);
    for (int p = 0; p < ex.P; ++p) {
      if (ex.sigma[p] != 0.0)
        launch_convert_add((const float*)ex.ylow[p], x[p], ex.sigma[p], y[p], ex.npsi[p], s);
      else
        launch_convert(1, ex.ylow[p], y[p], ex.npsi[p], s);
    }
  }
  IDMRG_HIP(hipGetLastError());
}

// Record what body(stream) launches into a HIP graph and instantiate it.  The
// launches go to the context's capture stream (the library's launchers read
// c->stream, which points there for the duration), so nothing runs now; the
// instance is replayed on the context stream.  Default priority, like every
// stream of the library.
template <typename F>
hipGraphExec_t capture_graph(idmrg_ctx* c, F&& body) {
  if (!c->cap) IDMRG_HIP(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
  const hipStream_t keep = c->stream;
  IDMRG_HIP(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
  c->stream = c->cap;
  hipGraph_t g = nullptr;
  try {
    body(c->cap);
  } catch (...) {
    c->stream = keep;
    (void)hipStreamEndCapture(c->cap, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  c->stream = keep;
  IDMRG_HIP(hipStreamEndCapture(c->cap, &g));
  hipGraphExec_t e = nullptr;
  const hipError_t r = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (r != hipSuccess) throw HipFailure(std::string("hipGraphInstantiate: ") + hipGetErrorString(r));
  return e;
}

// Instantiated graphs of one call; released after the stream has drained.
struct GraphSet {
  hipStream_t s;
  hipGraphExec_t ex[4] = {};
  explicit GraphSet(hipStream_t st) : s(st) {}
  ~GraphSet() {
    bool any = false;
    for (auto e : ex) any = any || e;
    if (!any) return;
    (void)hipStreamSynchronize(s);
    for (auto e : ex)
      if (e) (void)hipGraphExecDestroy(e);
  }
};

void check_nprob(int nprob) {
  if (nprob < 1 || nprob > 64) throw InvalidArg("nprob must be 1..64");
}

}  // namespace

// ------------------------------------------------------------------ context API

extern "C" int idmrg_create(idmrg_ctx** ctx, int device, void* hip_stream) {
  if (!ctx) return IDMRG_EINVAL;
  *ctx = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return IDMRG_EHIP;
  if (hipSetDevice(device) != hipSuccess) return IDMRG_EHIP;
  auto* c = new (std::nothrow) idmrg_ctx();
  if (!c) return IDMRG_ENOMEM;
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  *ctx = c;
  return IDMRG_OK;
}

extern "C" int idmrg_destroy(idmrg_ctx* c) {
  if (!c) return IDMRG_OK;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  if (c->plan.p) (void)hipFree(c->plan.p);
  for (auto& b : c->ws)
    if (b.p) (void)hipFree(b.p);
  if (c->pinned) (void)hipHostFree(c->pinned);
  for (auto& r : c->pending) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : c->pool) (void)hipEventDestroy(e);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  for (auto& row : c->tev)
    for (auto e : row)
      if (e) (void)hipEventDestroy(e);
  delete c;
  return IDMRG_OK;
}

extern "C" int idmrg_set_stream(idmrg_ctx* c, void* hip_stream) {
  if (!c) return IDMRG_EINVAL;
  (void)hipStreamSynchronize(c->stream);
  c->stream = (hipStream_t)hip_stream;
  return IDMRG_OK;
}

extern "C" int idmrg_profile(idmrg_ctx* c, int enable) {
  return guarded(c, [&]() {
    prof_collect(c);
    c->prof = enable != 0;
    if (enable)
      for (int k = 0; k < IDMRG_PROF_CLASSES; ++k) c->prof_n[k] = 0, c->prof_ms[k] = 0, c->prof_flops[k] = 0;
    return IDMRG_OK;
  });
}

extern "C" int idmrg_profile_get(idmrg_ctx* c, int cls, int64_t* launches, double* ms, double* flops) {
  return guarded(c, [&]() {
    if (cls < 0 || cls >= IDMRG_PROF_CLASSES || !launches || !ms || !flops) throw InvalidArg("bad profile query");
    prof_collect(c);
    *launches = c->prof_n[cls];
    *ms = c->prof_ms[cls];
    *flops = c->prof_flops[cls];
    return IDMRG_OK;
  });
}

extern "C" const char* idmrg_last_error(const idmrg_ctx* c) { return c ? c->err.c_str() : "null context"; }

extern "C" int64_t idmrg_psi_size(idmrg_leg A, idmrg_leg B, int32_t d, const int32_t* qp) {
  try {
    return psi_layout(make_leg(A, "A"), make_leg(B, "B"), make_qp(d, qp)).size;
  } catch (...) {
    return -1;
  }
}

extern "C" int64_t idmrg_envL_size(idmrg_leg A, int32_t dl, const int32_t* ql) {
  try {
    if (dl < 2 || !ql) return -1;
    return envL_layout(make_leg(A, "A"), std::vector<int>(ql, ql + dl)).size;
  } catch (...) {
    return -1;
  }
}

extern "C" int64_t idmrg_envR_size(idmrg_leg B, int32_t dr, const int32_t* qr) {
  try {
    if (dr < 2 || !qr) return -1;
    return envR_layout(make_leg(B, "B"), std::vector<int>(qr, qr + dr)).size;
  } catch (...) {
    return -1;
  }
}

extern "C" int64_t idmrg_U_size(idmrg_leg A, int32_t d, const int32_t* qp, idmrg_leg C) {
  try {
    return U_layout(make_leg(A, "A"), make_qp(d, qp), make_leg(C, "C")).size;
  } catch (...) {
    return -1;
  }
}

extern "C" int64_t idmrg_V_size(idmrg_leg B, int32_t d, const int32_t* qp, idmrg_leg C) {
  try {
    return V_layout(make_leg(B, "B"), make_qp(d, qp), make_leg(C, "C")).size;
  } catch (...) {
    return -1;
  }
}

extern "C" int idmrg_heff_work(const idmrg_heff* H, double* flops, double* bytes) {
  if (!H || !flops || !bytes) return IDMRG_EINVAL;
  try {
    const Mpo W1 = make_mpo(H->w1, "w1"), W2 = make_mpo(H->w2, "w2");
    heff_work(make_leg(H->left, "left"), make_leg(H->right, "right"), W1, W2, *flops, *bytes);
    return IDMRG_OK;
  } catch (...) {
    return IDMRG_EINVAL;
  }
}

// ------------------------------------------------------------------ heff_apply

extern "C" int heff_apply(idmrg_ctx* ctx, int nprob, const idmrg_heff* H, const double* const* x, double* const* y,
                          int prec) {
  return guarded(ctx, [&]() {
    check_nprob(nprob);
    if (!H || !x || !y) throw InvalidArg("null argument");
    std::vector<double*> xs(nprob), ys(nprob);
    for (int p = 0; p < nprob; ++p) {
      if (!x[p] || !y[p] || x[p] == y[p]) throw InvalidArg("x and y must be distinct device pointers");
      xs[p] = const_cast<double*>(x[p]);
      ys[p] = y[p];
    }
    HeffExec ex;
    heff_setup(ctx, ex, nprob, H, xs, ys, prec);
    heff_run(ctx, ex, xs, ys, nullptr);
    return IDMRG_OK;
  });
}

// ------------------------------------------------------------------ lanczos_solve_batch

extern "C" int lanczos_solve_batch(idmrg_ctx* ctx, int nprob, const idmrg_heff* H, double* const* psi,
                                   const idmrg_lanczos_opts* o, double* energy, idmrg_lanczos_info* info) {
  return guarded(ctx, [&]() {
    check_nprob(nprob);
    if (!H || !psi || !o || !energy || !info) throw InvalidArg("null argument");
    if (o->k_max < 1 || o->k_max > kLzMaxK) throw InvalidArg("k_max must be 1..1024");
    if (!(o->tol_E >= 0) || !(o->tol_res >= 0)) throw InvalidArg("tolerances must be >= 0");
    if (o->prec < 0 || o->prec > 2) throw InvalidArg("unknown precision policy");
    const int P = nprob;
    const int kmax = o->k_max;
    const int chunk = std::max(1, o->chunk > 0 ? o->chunk : 8);
    const bool mixed = o->prec != IDMRG_PREC_F64;
    hipStream_t s = ctx->stream;
    // sizes first (plan building validates everything)
    std::vector<int64_t> N(P);
    for (int p = 0; p < P; ++p) {
      if (!psi[p]) throw InvalidArg("null psi");
      N[p] = psi_layout(make_leg(H[p].left, "left"), make_leg(H[p].right, "right"),
                        make_mpo(H[p].w1, "w1").qp).size;
      if (N[p] == 0) throw InvalidArg("empty two-site space");
      check_dev(psi[p], N[p], 8, "psi");
    }
    // vectors: Q [kcap x N], w, v
    // every piece is a multiple of kLzAlign elements, so all rows start 2 KiB-aligned
    // (mixed precision also keeps the normalised start vector s0: the fidelity
    // of Eq. (12) is taken against the refined state that is returned)
    std::vector<int64_t> kcap(P), qoff(P), woff(P), voff(P), soff(P), ld(P);
    int64_t tot = 0;
    for (int p = 0; p < P; ++p) {
      kcap[p] = std::min<int64_t>(kmax, N[p]);
      ld[p] = (N[p] + kLzAlign - 1) / kLzAlign * kLzAlign;
      qoff[p] = tot;
      tot += kcap[p] * ld[p];
      woff[p] = tot;
      tot += ld[p];
      voff[p] = tot;
      tot += ld[p];
      soff[p] = tot;
      if (mixed) tot += ld[p];
    }
    double* V = (double*)ensure(ctx, ctx->ws[WS_LZ], tot * 8);
    const size_t nsm = (size_t)P * kmax;
    const size_t small_bytes =
        (size_t)P * (kmax + 1) * kLzBlocks * 8 + 4 * nsm * 8 + P * sizeof(LzCtrl) + P * 4 + 4096;
    char* sm = (char*)ensure(ctx, ctx->ws[WS_LZSMALL], small_bytes);
    double* partial = (double*)sm;
    double* alpha = partial + (size_t)P * kmax * kLzBlocks;
    double* beta = alpha + nsm;
    double* ritz = beta + nsm;
    double* coef = ritz + nsm;
    LzCtrl* ctrl = (LzCtrl*)(coef + nsm);
    double* pnorm = (double*)(ctrl + P);   // [P][kLzBlocks]
    int32_t* active = (int32_t*)(pnorm + (size_t)P * kLzBlocks);
    std::vector<double*> vv(P), ww(P);
    std::vector<LzProblem> probs(P);
    for (int p = 0; p < P; ++p) {
      vv[p] = V + voff[p];
      ww[p] = V + woff[p];
      probs[p] = LzProblem{N[p], ld[p], V + qoff[p], ww[p], vv[p], psi[p], mixed ? V + soff[p] : nullptr};
    }
    // The two plans use disjoint scratch buffers (T1, T3, plan), so setting up
    // the second never reallocates memory that the first has uploaded.
    HeffExec ex64, exlo;
    heff_setup(ctx, ex64, P, H, vv, ww, IDMRG_PREC_F64, &ctx->ws[WS_PLAN64]);
    if (mixed) heff_setup(ctx, exlo, P, H, vv, ww, o->prec, &ctx->ws[WS_PLANLOW]);
    char* dprob = (char*)ensure(ctx, ctx->ws[WS_MISC], P * (sizeof(LzProblem) + sizeof(LzCtrl) + 4) + 1024);
    LzProblem* dprobs = (LzProblem*)dprob;
    LzCtrl* hstage = (LzCtrl*)(dprob + ((P * sizeof(LzProblem) + 255) / 256) * 256);
    int32_t* astage = (int32_t*)((char*)hstage + ((P * sizeof(LzCtrl) + 255) / 256) * 256);
    sync(ctx);
    IDMRG_HIP(hipMemcpy(dprobs, probs.data(), P * sizeof(LzProblem), hipMemcpyHostToDevice));

    // Mixed precision: every outer pass is a Lanczos run whose first matvec is
    // FP64 (so alpha_0 and beta_0 are the exact Rayleigh quotient and residual
    // norm of the current vector) and whose later matvecs use the low-precision
    // policy; the pass's Ritz vector starts the next pass.  A pass that stops
    // at its first step (beta_0 <= tol_res) has converged in FP64.
    // (split-bf16: swept on the YC8 m = 2048 workload with the energy-shifted
    // copies, least Lanczos time per step; three passes per solve)
    const double lowE = o->prec == IDMRG_PREC_F32 ? 1e-9 : 1e-6;
    const double lowR = o->prec == IDMRG_PREC_F32 ? 1e-5 : 5e-5;
    const int k_inner = o->prec == IDMRG_PREC_F32 ? 70 : 100;
    const int max_outer = mixed ? 16 : 1;
    // Tile autotuning: the first matvecs of the precision that does most of the
    // work try one tiling variant each (identical results), then the fastest
    // variant of each stage is kept and remembered for this shape bucket.
    HeffExec& bulk = mixed ? exlo : ex64;
    bool tuned = !(bulk.need_tune[0] || bulk.need_tune[1]);
    int trial_next = 0;
    if (!tuned)
      for (auto& row : ctx->tev)
        for (auto& e : row)
          if (!e) IDMRG_HIP(hipEventCreate(&e));
    std::vector<int32_t> going(P, 1);
    std::vector<int> iters(P, 0), fp64mv(P, 0), reorths(P, 0);
    std::vector<LzCtrl> fin(P), out(P);
    std::vector<double> ov0(P, 0.0);
    GraphSet graphs(s);
    for (int outer = 0; outer < max_outer; ++outer) {
      std::vector<LzCtrl> hctrl(P);
      std::vector<int32_t> hact(P);
      int64_t maxk = 0;
      for (int p = 0; p < P; ++p) {
        LzCtrl z{};
        z.active = going[p];
        z.kcap = going[p] ? (int32_t)std::min<int64_t>(mixed && outer > 0 ? k_inner : kmax, kcap[p]) : 0;
        hctrl[p] = z;
        hact[p] = going[p];
        maxk = std::max<int64_t>(maxk, z.kcap);
      }
      sync(ctx);
      IDMRG_HIP(hipMemcpy(hstage, hctrl.data(), P * sizeof(LzCtrl), hipMemcpyHostToDevice));
      IDMRG_HIP(hipMemcpy(astage, hact.data(), P * 4, hipMemcpyHostToDevice));
      IDMRG_HIP(hipMemcpyAsync(ctrl, hstage, P * sizeof(LzCtrl), hipMemcpyDeviceToDevice, s));
      IDMRG_HIP(hipMemcpyAsync(active, astage, P * 4, hipMemcpyDeviceToDevice, s));
      lz_init(P, dprobs, ctrl, partial, kmax, s);
      if (outer == 0) {
        if (mixed)
          for (int p = 0; p < P; ++p)
            IDMRG_HIP(hipMemcpyAsync(probs[p].s0, vv[p], ld[p] * 8, hipMemcpyDeviceToDevice, s));
        std::vector<LzCtrl> chk(P);
        IDMRG_HIP(hipMemcpyAsync(chk.data(), ctrl, P * sizeof(LzCtrl), hipMemcpyDeviceToHost, s));
        sync(ctx);
        for (int p = 0; p < P; ++p)
          if (!(chk[p].norm0 > 0.0) || !std::isfinite(chk[p].norm0))
            throw InvalidArg("start vector has zero or non-finite norm (problem " + std::to_string(p) + ")");
      }
      const double tolE = mixed ? std::max(o->tol_E, lowE) : o->tol_E;
      const double tolR = mixed ? std::max(o->tol_res, lowR) : o->tol_res;
      const double tolF = mixed ? o->tol_res : 0.0;
      // refinement passes reduce the exact residual by a fixed factor each
      const double relF = (mixed && outer > 0) ? (o->prec == IDMRG_PREC_F32 ? 1e-4 : 2e-4) : 0.0;
      std::vector<int32_t> act(P);
      // one iteration: matvec (FP64 for the first of a mixed pass) and the vector work
      auto iteration = [&](int64_t i, int trial, hipStream_t st) {
        HeffExec& e = (!mixed || i == 0) ? ex64 : exlo;
        heff_run(ctx, e, vv, ww, active, trial);
        Prof pr(ctx, 4, 0.0);
        lz_iteration_tail(P, dprobs, ctrl, active, alpha, beta, ritz, coef, partial, pnorm, kmax, tolE, tolR, tolF,
                          relF, o->cgs2 ? 1 : 0, st);
      };
      for (int64_t it = 0; it < maxk;) {
        if (o->graph && tuned && !ctx->prof && it + chunk <= maxk) {
          // a full chunk as one graph launch; the launches depend only on whether the chunk
          // opens a mixed pass (FP64 first matvec) and on the pass's tolerances (outer > 0)
          const int key = (mixed && it == 0 ? 1 : 0) + (outer > 0 ? 2 : 0);
          if (!graphs.ex[key]) {
            const int64_t i0 = it;
            graphs.ex[key] = capture_graph(ctx, [&](hipStream_t cs) {
              for (int k = 0; k < chunk; ++k) iteration(i0 + k, -1, cs);
            });
          }
          IDMRG_HIP(hipGraphLaunch(graphs.ex[key], s));
          it += chunk;
        } else {
          for (int k = 0; k < chunk && it < maxk; ++k, ++it) {
            HeffExec& e = (!mixed || it == 0) ? ex64 : exlo;
            const int trial = (!tuned && &e == &bulk && trial_next < bulk.nvar) ? trial_next++ : -1;
            iteration(it, trial, s);
          }
        }
        IDMRG_HIP(hipMemcpyAsync(act.data(), active, P * 4, hipMemcpyDeviceToHost, s));
        sync(ctx);
        if (!tuned && trial_next == bulk.nvar) {
          tune_resolve(ctx, bulk, trial_next);
          tuned = true;
        }
        if (std::all_of(act.begin(), act.end(), [](int32_t a) { return a == 0; })) break;
      }
      if (!tuned && trial_next > 0) {   // the pass ended before every variant was tried
        tune_resolve(ctx, bulk, trial_next);
        tuned = true;
      }
      lz_finish(P, dprobs, ctrl, ritz, partial, kmax, s);
      IDMRG_HIP(hipMemcpyAsync(out.data(), ctrl, P * sizeof(LzCtrl), hipMemcpyDeviceToHost, s));
      sync(ctx);
      for (int p = 0; p < P; ++p) {
        if (!going[p]) continue;
        iters[p] += out[p].iters;
        reorths[p] += out[p].reorths;
        fp64mv[p] += 1;
        if (outer == 0) ov0[p] = out[p].overlap0;
        fin[p] = out[p];
        if (!mixed || (out[p].iters == 1 && out[p].converged)) going[p] = 0;
      }
      if (std::all_of(going.begin(), going.end(), [](int32_t g) { return g == 0; })) break;
    }
    if (mixed) {
      // |<start, psi>| against the returned (refined) state
      lz_overlap(P, dprobs, ctrl, partial, kmax, s);
      IDMRG_HIP(hipMemcpyAsync(out.data(), ctrl, P * sizeof(LzCtrl), hipMemcpyDeviceToHost, s));
      sync(ctx);
      for (int p = 0; p < P; ++p) ov0[p] = out[p].overlap0;
    }
    if (!mixed) {
      // FP64 residual of the result: w = H psi (v holds psi after lz_finish)
      heff_run(ctx, ex64, vv, ww, nullptr);
      lz_residual(P, dprobs, ctrl, partial, kmax, s);
      IDMRG_HIP(hipMemcpyAsync(out.data(), ctrl, P * sizeof(LzCtrl), hipMemcpyDeviceToHost, s));
      sync(ctx);
      for (int p = 0; p < P; ++p) fin[p].residual = out[p].residual;
    }
    int rc = IDMRG_OK;
    for (int p = 0; p < P; ++p) {
      energy[p] = fin[p].theta;
      info[p].overlap0 = ov0[p];
      info[p].iters = iters[p];
      info[p].converged = mixed ? (going[p] ? 0 : 1) : fin[p].converged;
      info[p].fp64_matvecs = mixed ? fp64mv[p] : 0;
      info[p].flags = fin[p].flags;
      info[p].reorth_passes = reorths[p];
      info[p].reserved = 0;
      info[p].residual = fin[p].residual;
      if (!std::isfinite(fin[p].theta) || !std::isfinite(fin[p].residual)) {
        ctx->err = "non-finite energy or residual (problem " + std::to_string(p) + ")";
        return IDMRG_ENUMERIC;
      }
      if (!info[p].converged) rc = IDMRG_WARN_NOCONV;
    }
    return rc;
  });
}
// ------------------------------------------------------------------ truncate_twosite

extern "C" int truncate_twosite(idmrg_ctx* ctx, int nprob, int32_t d, const int32_t* qp_in, int32_t m_max,
                                double lam_floor, double deg_rel, idmrg_trunc* t) {
  return guarded(ctx, [&]() {
    check_nprob(nprob);
    if (!t || m_max < 1 || !(lam_floor >= 0) || !(deg_rel >= 0)) throw InvalidArg("bad truncation arguments");
    const std::vector<int> qp = make_qp(d, qp_in);
    const int P = nprob;
    hipStream_t s = ctx->stream;
    struct Sec { int q, r, c; std::vector<std::tuple<int, int, int>> rows, cols; int64_t m, x, g, u, v, sv; };
    std::vector<std::vector<Sec>> secs(P);
    std::vector<Leg> A(P), B(P);
    std::vector<PsiLayout> X(P);
    int64_t nM = 0, nX = 0, nG = 0, nU = 0, nV = 0, nS = 0;
    int svd_sweeps = 0, svd_conv = 1;
    std::vector<int32_t> completed(P, 1);
    MixList gather;
    std::vector<SvdTask> svd;
    std::vector<SelTask> sel;
    std::vector<SelSector> ssec;
    int ncand_tot = 0;
    for (int p = 0; p < P; ++p) {
      if (!t[p].psi) throw InvalidArg("null psi");
      A[p] = make_leg(t[p].left, "trunc.left");
      B[p] = make_leg(t[p].right, "trunc.right");
      X[p] = psi_layout(A[p], B[p], qp);
      std::map<int, Sec> byq;
      for (int a = 0; a < A[p].n(); ++a)
        for (int s1 = 0; s1 < d; ++s1) {
          Sec& S = byq[A[p].q[a] + qp[s1]];
          S.rows.emplace_back(a, s1, S.r);
          S.r += A[p].dim[a];
        }
      for (int s2 = 0; s2 < d; ++s2)
        for (int b = 0; b < B[p].n(); ++b) {
          Sec& S = byq[B[p].q[b] - qp[s2]];
          S.cols.emplace_back(s2, b, S.c);
          S.c += B[p].dim[b];
        }
      SelTask st{};
      st.sec0 = (int)ssec.size();
      st.cand0 = ncand_tot;
      st.m_max = m_max;
      st.prob = p;
      st.lam_floor = lam_floor;
      st.deg_rel = deg_rel;
      for (auto& kv : byq) {
        Sec S = kv.second;
        S.q = kv.first;
        if (S.r == 0 || S.c == 0) continue;
        const int n = std::min(S.r, S.c), pp = std::max(S.r, S.c);
        if (n > 4096 || pp > 8192)
          throw InvalidArg("centre sector larger than 4096 x 8192 states is not supported");
        S.m = nM; nM += (int64_t)S.r * S.c;
        S.x = nX; nX += (int64_t)n * pp;
        S.g = nG; nG += (int64_t)n * n;
        S.u = nU; nU += (int64_t)S.r * n;
        S.v = nV; nV += (int64_t)S.c * n;
        S.sv = nS; nS += n;
        for (auto& rw : S.rows)
          for (auto& cl : S.cols) {
            const int a = std::get<0>(rw), s1 = std::get<1>(rw), ro = std::get<2>(rw);
            const int s2 = std::get<0>(cl), b = std::get<1>(cl), co = std::get<2>(cl);
            const int xi = X[p].find(a, s1, s2);
            if (xi < 0 || X[p].blk[xi].b != b) throw InvalidArg("internal: truncation block bookkeeping");
            MixTask m{};
            m.rows = A[p].dim[a]; m.cols = B[p].dim[b]; m.ldd = S.c; m.prob = p; m.dbase = 1;
            m.doff = S.m + (int64_t)ro * S.c + co;
            MixSrc sr{};
            sr.coef = 1.0; sr.base = 0; sr.off = X[p].blk[xi].off; sr.ld = B[p].dim[b];
            gather.add(m, {sr});
          }
        SvdTask sv{};
        sv.r = S.r; sv.c = S.c; sv.prob = p;
        sv.m_off = S.m; sv.x_off = S.x; sv.g_off = S.g; sv.u_off = S.u; sv.v_off = S.v; sv.s_off = S.sv;
        svd.push_back(sv);
        SelSector se{};
        se.charge = S.q; se.n = n; se.cand0 = ncand_tot; se.s_off = S.sv;
        ssec.push_back(se);
        ncand_tot += n;
        st.ncand += n;
        st.nsec += 1;
        secs[p].push_back(S);
      }
      if (st.ncand > 8192) throw InvalidArg("more than 8192 singular values per problem is not supported");
      if (st.ncand == 0) throw InvalidArg("two-site state has no centre sector");
      sel.push_back(st);
    }
    // S values of all problems live in one array: make s_off global
    // (each problem's sectors were given offsets into its own region; regions are disjoint)
    char* ws = (char*)ensure(ctx, ctx->ws[WS_SVD], (nM + nX + nG + nU + nV + nS + 6 * 64) * 8);
    double* dM = (double*)ws;
    double* dX = dM + nM + 64;
    double* dG = dX + nX + 64;
    double* dU = dG + nG + 64;
    double* dV = dU + nU + 64;
    double* dS = dV + nV + 64;
    const size_t selb = (size_t)ncand_tot * (4 + 8) + ssec.size() * 4 + P * 32 + 4096;
    char* sw = (char*)ensure(ctx, ctx->ws[WS_SEL], selb);
    int32_t* colmap = (int32_t*)sw;
    double* lam_sel = (double*)(sw + ((size_t)ncand_tot * 4 + 255) / 256 * 256);
    int32_t* kept = (int32_t*)((char*)lam_sel + ((size_t)ncand_tot * 8 + 255) / 256 * 256);
    double* scal = (double*)((char*)kept + (ssec.size() * 4 + 255) / 256 * 256);
    {
      std::vector<int64_t> sz((size_t)P * kNumBases, -1);
      for (int p = 0; p < P; ++p) {
        sz[(size_t)p * kNumBases + 0] = X[p].size;
        sz[(size_t)p * kNumBases + 1] = nM;
        check_dev(t[p].psi, X[p].size, 8, "psi");
      }
      check_mix(gather, sz, "truncation gather");
    }
    std::vector<void*> hb((size_t)P * kNumBases, nullptr);
    for (int p = 0; p < P; ++p) {
      void** b = &hb[(size_t)p * kNumBases];
      b[0] = (void*)t[p].psi; b[1] = dM; b[2] = dX; b[3] = dG; b[4] = dU; b[5] = dV; b[6] = dS;
    }
    std::vector<int32_t> sweeps(svd.size(), 0);
    Packer pk;
    const size_t a1 = pk.add(gather.t), a2 = pk.add(gather.src), a3 = pk.add(svd), a4 = pk.add(sel),
                 a5 = pk.add(ssec), a6 = pk.add(hb), a7 = pk.add(sweeps);
    char* dev = upload(ctx, pk);
    {
      Prof pr(ctx, 6, 0.0);
      launch_mix(0, 0, (MixTask*)(dev + a1), (MixSrc*)(dev + a2), (int)gather.t.size(), gather.tiles,
                 (void**)(dev + a6), nullptr, s);
    }
    {
      Prof pr(ctx, 5, 0.0);
      BjScratch scr;
      int pmax = 1;
      for (const auto& sv : svd) pmax = std::max(pmax, std::max(sv.r, sv.c));
      scr.tol = std::max(1e-15, 4.4e-16 * std::sqrt((double)pmax));
      // null rows: at most 1e-15 .. 1e-14 of their block's norm (rounding residue); never
      // above lam_floor, so that a null row never ranks as a nonzero value unless lam_floor
      // itself is below 1e-15
      scr.zero_rel = std::min(std::max(lam_floor, 1e-15), 1e-14);
      auto up = [&](const std::vector<char>& h) -> char* {
        char* d = (char*)ensure(ctx, ctx->ws[WS_READ], h.size());
        sync(ctx);
        IDMRG_HIP(hipMemcpy(d, h.data(), h.size(), hipMemcpyHostToDevice));
        return d;
      };
      // Null rows (sigma <= zero_rel |M_q|_F) need a completed direction only if the
      // selection can keep one.  Zero-weight states are kept only when every candidate is
      // (m_max >= candidates); otherwise a null row is kept only if it ranks as a nonzero
      // value, which needs lam_floor < zero_rel.  "above" counts conservatively the rows
      // with sigma / |sigma| above zero_rel (1 + 1e-9), which no null row reaches: when all
      // of the kept states are among them, no completion is needed.
      scr.need_completion = [&](std::vector<int32_t>& complete) {
        std::vector<double> hS(nS);
        IDMRG_HIP(hipMemcpyAsync(hS.data(), dS, nS * 8, hipMemcpyDeviceToHost, s));
        sync(ctx);
        std::vector<double> tot(P, 0.0);
        std::vector<int64_t> cand(P, 0), above(P, 0);
        for (const auto& sv : svd) {
          const int n = std::min(sv.r, sv.c);
          cand[sv.prob] += n;
          for (int i = 0; i < n; ++i) tot[sv.prob] += hS[sv.s_off + i] * hS[sv.s_off + i];
        }
        const double thr = scr.zero_rel * (1.0 + 1e-9);
        for (const auto& sv : svd) {
          const int n = std::min(sv.r, sv.c);
          const double cut = thr * std::sqrt(tot[sv.prob]);
          for (int i = 0; i < n; ++i) above[sv.prob] += hS[sv.s_off + i] > cut;
        }
        for (int pr = 0; pr < P; ++pr) {
          const bool all_kept = m_max >= cand[pr];
          const bool null_may_rank = lam_floor < scr.zero_rel;
          completed[pr] = !(tot[pr] > 0.0 && (all_kept ? above[pr] >= cand[pr]
                                                       : (!null_may_rank || above[pr] >= m_max)));
        }
        for (size_t m = 0; m < svd.size(); ++m) complete[m] = completed[svd[m].prob];
      };
      bj_svd(svd, (void**)(dev + a6), (SvdTask*)(dev + a3), scr, s, up,
             [&](size_t b) { return (char*)ensure(ctx, ctx->ws[WS_BJ], b); }, [&]() { sync(ctx); });
      (void)a7;
      svd_sweeps = scr.sweeps;
      svd_conv = scr.converged;
    }
    {
      Prof pr(ctx, 6, 0.0);
      launch_select((SelTask*)(dev + a4), (int)sel.size(), (SelSector*)(dev + a5), dS, kept, colmap, lam_sel, scal,
                    s);
    }
    IDMRG_HIP(hipGetLastError());
    std::vector<int32_t> hkept(ssec.size());
    std::vector<double> hscal(4 * (size_t)P);
    IDMRG_HIP(hipMemcpyAsync(hkept.data(), kept, hkept.size() * 4, hipMemcpyDeviceToHost, s));
    IDMRG_HIP(hipMemcpyAsync(hscal.data(), scal, hscal.size() * 8, hipMemcpyDeviceToHost, s));
    sync(ctx);
    // outputs
    ScaleList outl;
    std::vector<void*> ob((size_t)P * kNumBases, nullptr);
    for (int p = 0; p < P; ++p) {
      const SelTask& st = sel[p];
      Leg C;
      std::vector<int> which;
      for (int k = 0; k < st.nsec; ++k)
        if (hkept[st.sec0 + k] > 0) {
          C.q.push_back(ssec[st.sec0 + k].charge);
          C.dim.push_back(hkept[st.sec0 + k]);
          which.push_back(k);
        }
      if (C.n() > t[p].cap_sec || !t[p].q_out || !t[p].dim_out) throw InvalidArg("new-leg capacity too small");
      const IsoLayout U = U_layout(A[p], qp, C), Vl = V_layout(B[p], qp, C);
      if (U.size > t[p].cap_U || Vl.size > t[p].cap_V || C.total() > t[p].cap_lam)
        throw InvalidArg("output capacity too small (U, V or lambda)");
      if (!t[p].U || !t[p].V || !t[p].lambda) throw InvalidArg("null output buffer");
      void** b = &ob[(size_t)p * kNumBases];
      b[0] = dU; b[1] = dV; b[2] = lam_sel; b[3] = t[p].U; b[4] = t[p].V; b[5] = t[p].lambda;
      int64_t loff = 0;
      for (int ci = 0; ci < C.n(); ++ci) {
        const Sec& S = secs[p][which[ci]];
        const SelSector& se = ssec[st.sec0 + which[ci]];
        const int n = se.n, k = C.dim[ci];
        if (U.rows[ci] != S.r || Vl.rows[ci] != S.c) throw InvalidArg("internal: isometry row mismatch");
        ScaleTask a{};
        a.rows = S.r; a.cols = k; a.lds = n; a.ldd = k; a.prob = p; a.sbase = 0; a.dbase = 3; a.rbase = -1;
        a.cbase = -1; a.colmap = se.cand0; a.soff = S.u; a.doff = U.off[ci];
        outl.add(a);
        ScaleTask v = a;
        v.rows = S.c; v.sbase = 1; v.dbase = 4; v.soff = S.v; v.doff = Vl.off[ci];
        outl.add(v);
        ScaleTask l{};
        l.rows = 1; l.cols = k; l.lds = k; l.ldd = k; l.prob = p; l.sbase = 2; l.dbase = 5; l.rbase = -1;
        l.cbase = -1; l.colmap = -1; l.soff = se.cand0; l.doff = loff;
        outl.add(l);
        loff += k;
        t[p].q_out[ci] = C.q[ci];
        t[p].dim_out[ci] = k;
      }
      t[p].nsec_out = C.n();
      t[p].eps = hscal[4 * p + 0];
      t[p].eps_prime = hscal[4 * p + 1];
      t[p].cut_gap = hscal[4 * p + 2];
      t[p].m_kept = (int32_t)hscal[4 * p + 3];
      t[p].svd_sweeps = svd_sweeps;
      t[p].svd_converged = svd_conv;
      t[p].null_completed = completed[p];
      t[p].reserved = 0;
    }
    {
      std::vector<int64_t> sz((size_t)P * kNumBases, -1);
      for (int p = 0; p < P; ++p) {
        int64_t* z = &sz[(size_t)p * kNumBases];
        z[0] = nU; z[1] = nV; z[2] = ncand_tot; z[3] = t[p].cap_U; z[4] = t[p].cap_V; z[5] = t[p].cap_lam;
        check_dev(t[p].U, t[p].cap_U, 8, "U");
        check_dev(t[p].V, t[p].cap_V, 8, "V");
        check_dev(t[p].lambda, t[p].cap_lam, 8, "lambda");
      }
      check_scale(outl, sz, "truncation output", ncand_tot);
    }
    Packer pk2;
    const size_t b1 = pk2.add(outl.t), b2 = pk2.add(ob);
    char* dev2 = upload(ctx, pk2);
    {
      Prof pr(ctx, 6, 0.0);
      launch_scale((ScaleTask*)(dev2 + b1), colmap, (int)outl.t.size(), outl.tiles, 0.0, (void**)(dev2 + b2), s);
    }
    IDMRG_HIP(hipGetLastError());
    sync(ctx);
    for (int p = 0; p < P; ++p)
      if (!std::isfinite(t[p].eps)) {
        ctx->err = "non-finite singular values";
        return IDMRG_ENUMERIC;
      }
    if (!svd_conv) {
      ctx->err = "Jacobi SVD did not converge in " + std::to_string(svd_sweeps) + " sweeps";
      return IDMRG_WARN_NOCONV;
    }
    return IDMRG_OK;
  });
}

// ------------------------------------------------------------------ update_env

extern "C" int update_env(idmrg_ctx* ctx, int nprob, int side, const idmrg_env_update* u) {
  return guarded(ctx, [&]() {
    check_nprob(nprob);
    if (!u || (side != IDMRG_LEFT && side != IDMRG_RIGHT)) throw InvalidArg("bad update_env arguments");
    const int P = nprob;
    EnvPlan plan;
    std::vector<int64_t> sz((size_t)P * kNumBases, -1);
    for (int p = 0; p < P; ++p) {
      if (!u[p].env_old || !u[p].iso || !u[p].env_new) throw InvalidArg("null buffer in idmrg_env_update");
      const Leg O = make_leg(u[p].old_leg, "env.old_leg"), C = make_leg(u[p].new_leg, "env.new_leg");
      const Mpo W = make_mpo(u[p].w, "env.w");
      int64_t* z = &sz[(size_t)p * kNumBases];
      if (side == IDMRG_LEFT) {
        build_envL(plan, p, O, C, W);
        z[0] = envL_layout(O, W.ql).size; z[1] = U_layout(O, W.qp, C).size; z[2] = envL_layout(C, W.qr).size;
      } else {
        build_envR(plan, p, O, C, W);
        z[0] = envR_layout(O, W.qr).size; z[1] = V_layout(O, W.qp, C).size; z[2] = envR_layout(C, W.ql).size;
      }
      z[3] = plan.n_T1[p]; z[4] = plan.n_T2[p];
      check_dev(u[p].env_old, z[0], 8, "env_old");
      check_dev(u[p].iso, z[1], 8, "iso");
      check_dev(u[p].env_new, z[2], 8, "env_new");
    }
    check_gemm(plan.ga, side == IDMRG_LEFT ? 0 : 2, sz, "env stage a");
    check_mix(plan.mix, sz, "env mix");
    check_gemm(plan.gc, side == IDMRG_LEFT ? 2 : 0, sz, "env stage c");
    int64_t n1 = 0, n2 = 0;
    std::vector<int64_t> o1(P), o2(P);
    for (int p = 0; p < P; ++p) {
      o1[p] = n1; n1 += plan.n_T1[p] + 64;
      o2[p] = n2; n2 += plan.n_T2[p] + 64;
    }
    double* ws = (double*)ensure(ctx, ctx->ws[WS_ENV], (n1 + n2) * 8);
    std::vector<void*> hb((size_t)P * kNumBases, nullptr);
    for (int p = 0; p < P; ++p) {
      void** b = &hb[(size_t)p * kNumBases];
      b[0] = (void*)u[p].env_old; b[1] = (void*)u[p].iso; b[2] = u[p].env_new;
      b[3] = ws + o1[p]; b[4] = ws + n1 + o2[p];
    }
    Packer pk;
    const size_t a1 = pk.add(plan.ga.t), a2 = pk.add(plan.mix.t), a3 = pk.add(plan.mix.src), a4 = pk.add(plan.gc.t),
                 a5 = pk.add(hb);
    char* dev = upload(ctx, pk);
    void** bases = (void**)(dev + a5);
    hipStream_t s = ctx->stream;
    Prof pr(ctx, 7, plan.ga.flops() + plan.gc.flops() + plan.mix.flops());
    launch_gemm(Prec::F64, side == IDMRG_LEFT ? 0 : 2, (GemmTask*)(dev + a1), (int)plan.ga.t.size(), plan.ga.tiles,
                bases, nullptr, s);
    launch_mix(0, 0, (MixTask*)(dev + a2), (MixSrc*)(dev + a3), (int)plan.mix.t.size(), plan.mix.tiles, bases,
               nullptr, s);
    launch_gemm(Prec::F64, side == IDMRG_LEFT ? 2 : 0, (GemmTask*)(dev + a4), (int)plan.gc.t.size(), plan.gc.tiles,
                bases, nullptr, s);
    IDMRG_HIP(hipGetLastError());
    return IDMRG_OK;
  });
}

// ------------------------------------------------------------------ predict_wavefunction

extern "C" int predict_wavefunction(idmrg_ctx* ctx, int nprob, int32_t d, const int32_t* qp_in, double lam_floor,
                                    const idmrg_predict* pr) {
  return guarded(ctx, [&]() {
    check_nprob(nprob);
    if (!pr || !(lam_floor >= 0)) throw InvalidArg("bad predict arguments");
    const std::vector<int> qp = make_qp(d, qp_in);
    const int P = nprob;
    PredictPlan plan;
    std::vector<int64_t> sz((size_t)P * kNumBases, -1);
    for (int p = 0; p < P; ++p) {
      if (!pr[p].lam_i || !pr[p].V_i || !pr[p].lam_prev || !pr[p].U_ip1 || !pr[p].lam_ip1 || !pr[p].psi)
        throw InvalidArg("null buffer in idmrg_predict");
      const Leg Aa = make_leg(pr[p].leg_a, "leg_a"), Bt = make_leg(pr[p].leg_beta, "leg_beta"),
                Bb = make_leg(pr[p].leg_b, "leg_b");
      build_predict(plan, p, Aa, Bt, Bb, qp);
      int64_t* z = &sz[(size_t)p * kNumBases];
      z[0] = Aa.total(); z[1] = z[6] = V_layout(Bt, qp, Aa).size; z[2] = Bt.total();
      z[3] = z[7] = U_layout(Bt, qp, Bb).size; z[4] = Bb.total(); z[5] = psi_layout(Aa, Bb, qp).size;
      check_dev(pr[p].lam_i, z[0], 8, "lam_i");
      check_dev(pr[p].V_i, z[1], 8, "V_i");
      check_dev(pr[p].lam_prev, z[2], 8, "lam_prev");
      check_dev(pr[p].U_ip1, z[3], 8, "U_ip1");
      check_dev(pr[p].lam_ip1, z[4], 8, "lam_ip1");
      check_dev(pr[p].psi, z[5], 8, "psi");
    }
    check_scale(plan.scale, sz, "predict scale", 0);
    check_gemm(plan.g, 2, sz, "predict gemm");
    int64_t n = 0;
    std::vector<int64_t> ov(P), ou(P);
    for (int p = 0; p < P; ++p) {
      ov[p] = n; n += plan.n_Vs[p] + 64;
      ou[p] = n; n += plan.n_Us[p] + 64;
    }
    double* ws = (double*)ensure(ctx, ctx->ws[WS_PRED], n * 8);
    std::vector<void*> hb((size_t)P * kNumBases, nullptr);
    for (int p = 0; p < P; ++p) {
      void** b = &hb[(size_t)p * kNumBases];
      b[0] = (void*)pr[p].lam_i; b[1] = (void*)pr[p].V_i; b[2] = (void*)pr[p].lam_prev; b[3] = (void*)pr[p].U_ip1;
      b[4] = (void*)pr[p].lam_ip1; b[5] = pr[p].psi; b[6] = ws + ov[p]; b[7] = ws + ou[p];
    }
    Packer pk;
    const size_t a1 = pk.add(plan.scale.t), a2 = pk.add(plan.g.t), a3 = pk.add(hb);
    char* dev = upload(ctx, pk);
    void** bases = (void**)(dev + a3);
    Prof pr(ctx, 8, plan.g.flops());
    launch_scale((ScaleTask*)(dev + a1), nullptr, (int)plan.scale.t.size(), plan.scale.tiles, lam_floor, bases,
                 ctx->stream);
    launch_gemm(Prec::F64, 2, (GemmTask*)(dev + a2), (int)plan.g.t.size(), plan.g.tiles, bases, nullptr, ctx->stream);
    IDMRG_HIP(hipGetLastError());
    return IDMRG_OK;
  });
}
