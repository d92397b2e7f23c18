// Host-side layouts and work-plan builders.  See plan.h and idmrg.h for the
// storage orders; the contractions are those of the paper's Step 3 (H_eff,
// Fig. 2(b)), Step 6 (Eqs. (4), (5)) and Step 3' (Eq. (10)).
#include <climits>
#include "plan.h"

#include <algorithm>
#include <cstring>
#include <cmath>

namespace idmrg {

int Leg::find(int charge) const {
  auto it = std::lower_bound(q.begin(), q.end(), charge);
  if (it == q.end() || *it != charge) return -1;
  return (int)(it - q.begin());
}

int64_t Leg::total() const {
  int64_t s = 0;
  for (int x : dim) s += x;
  return s;
}

Leg make_leg(const idmrg_leg& l, const char* what) {
  if (l.nsec < 1 || !l.q || !l.dim) throw InvalidArg(std::string(what) + ": empty leg");
  Leg g;
  for (int k = 0; k < l.nsec; ++k) {
    if (l.dim[k] < 1) throw InvalidArg(std::string(what) + ": sector dimension < 1");
    if (k > 0 && l.q[k] <= l.q[k - 1]) throw InvalidArg(std::string(what) + ": charges not strictly ascending");
    g.q.push_back(l.q[k]);
    g.dim.push_back(l.dim[k]);
  }
  return g;
}

std::vector<int> make_qp(int d, const int32_t* qp) {
  if (d < 1 || d > 16 || !qp) throw InvalidArg("local dimension must be 1..16 with charges");
  return std::vector<int>(qp, qp + d);
}

Mpo make_mpo(const idmrg_mpo* m, const char* what) {
  if (!m || !m->w || !m->ql || !m->qr || !m->qp) throw InvalidArg(std::string(what) + ": null MPO field");
  if (m->dl < 2 || m->dr < 2 || m->d < 1 || m->d > 16) throw InvalidArg(std::string(what) + ": bad MPO shape");
  Mpo o;
  o.dl = m->dl;
  o.dr = m->dr;
  o.d = m->d;
  o.w.assign(m->w, m->w + (int64_t)m->dl * m->dr * m->d * m->d);
  o.ql.assign(m->ql, m->ql + m->dl);
  o.qr.assign(m->qr, m->qr + m->dr);
  o.qp.assign(m->qp, m->qp + m->d);
  for (int a = 0; a < o.dl; ++a)
    for (int b = 0; b < o.dr; ++b)
      for (int s = 0; s < o.d; ++s)
        for (int t = 0; t < o.d; ++t) {
          const double v = o.at(a, b, s, t);
          if (!std::isfinite(v)) throw InvalidArg(std::string(what) + ": non-finite MPO entry");
          if (v != 0.0 && o.qp[s] - o.qp[t] != o.qr[b] - o.ql[a])
            throw InvalidArg(std::string(what) + ": MPO entry violates charge conservation");
        }
  for (int s = 0; s < o.d; ++s)
    for (int t = 0; t < o.d; ++t) {
      const double id = s == t ? 1.0 : 0.0;
      if (o.at(0, 0, s, t) != id || o.at(o.dl - 1, o.dr - 1, s, t) != id)
        throw InvalidArg(std::string(what) + ": W[0][0] and W[D-1][D-1] must be the identity");
    }
  if (o.ql[0] != 0 || o.qr[0] != 0 || o.ql[o.dl - 1] != 0 || o.qr[o.dr - 1] != 0)
    throw InvalidArg(std::string(what) + ": complete/identity channels must carry charge 0");
  return o;
}

// ------------------------------------------------------------------ layouts

PsiLayout psi_layout(const Leg& A, const Leg& B, const std::vector<int>& qp) {
  PsiLayout L;
  const int d = (int)qp.size();
  L.b_first.assign(B.n(), -1);
  L.b_rows.assign(B.n(), 0);
  for (int b = 0; b < B.n(); ++b)
    for (int a = 0; a < A.n(); ++a)
      for (int s1 = 0; s1 < d; ++s1)
        for (int s2 = 0; s2 < d; ++s2) {
          if (A.q[a] + qp[s1] + qp[s2] != B.q[b]) continue;
          PsiLayout::Blk k{b, a, s1, s2, L.size, A.dim[a], B.dim[b]};
          if (L.b_first[b] < 0) L.b_first[b] = L.size;
          L.b_rows[b] += A.dim[a];
          L.index[PsiLayout::key(a, s1, s2)] = (int)L.blk.size();
          L.blk.push_back(k);
          L.size += (int64_t)A.dim[a] * B.dim[b];
        }
  return L;
}

EnvLLayout envL_layout(const Leg& A, const std::vector<int>& dq) {
  EnvLLayout L;
  const int D = (int)dq.size();
  L.stack_off.assign(A.n(), 0);
  L.rows.assign(A.n(), 0);
  L.row_off.assign(A.n(), std::vector<int>(D, -1));
  L.a_out.assign(A.n(), std::vector<int>(D, -1));
  for (int ac = 0; ac < A.n(); ++ac) {
    L.stack_off[ac] = L.size;
    int r = 0;
    for (int w = 0; w < D - 1; ++w) {
      const int ar = A.find(A.q[ac] + dq[w]);
      if (ar < 0) continue;
      L.row_off[ac][w] = r;
      L.a_out[ac][w] = ar;
      r += A.dim[ar];
    }
    L.rows[ac] = r;
    L.size += (int64_t)r * A.dim[ac];
  }
  return L;
}

EnvRLayout envR_layout(const Leg& B, const std::vector<int>& dq) {
  EnvRLayout L;
  const int D = (int)dq.size();
  L.off.assign(B.n(), 0);
  L.K.assign(B.n(), 0);
  L.col_off.assign(B.n(), std::vector<int>(D, -1));
  L.b_in.assign(B.n(), std::vector<int>(D, -1));
  for (int b = 0; b < B.n(); ++b) {
    L.off[b] = L.size;
    int k = 0;
    for (int w = 1; w < D; ++w) {
      const int bi = B.find(B.q[b] - dq[w]);
      if (bi < 0) continue;
      L.col_off[b][w] = k;
      L.b_in[b][w] = bi;
      k += B.dim[bi];
    }
    L.K[b] = k;
    L.size += (int64_t)B.dim[b] * k;
  }
  return L;
}

int IsoLayout::row_of(int c, int sec, int s) const {
  for (const Grp& g : grp[c])
    if (g.sec == sec && g.s == s) return g.row;
  return -1;
}

IsoLayout U_layout(const Leg& A, const std::vector<int>& qp, const Leg& C) {
  IsoLayout L;
  const int d = (int)qp.size();
  L.off.assign(C.n(), 0);
  L.rows.assign(C.n(), 0);
  L.grp.assign(C.n(), {});
  for (int c = 0; c < C.n(); ++c) {
    L.off[c] = L.size;
    int r = 0;
    for (int a = 0; a < A.n(); ++a)
      for (int s = 0; s < d; ++s)
        if (A.q[a] + qp[s] == C.q[c]) {
          L.grp[c].push_back({a, s, r, A.dim[a]});
          r += A.dim[a];
        }
    L.rows[c] = r;
    L.size += (int64_t)r * C.dim[c];
  }
  return L;
}

IsoLayout V_layout(const Leg& B, const std::vector<int>& qp, const Leg& C) {
  IsoLayout L;
  const int d = (int)qp.size();
  L.off.assign(C.n(), 0);
  L.rows.assign(C.n(), 0);
  L.grp.assign(C.n(), {});
  for (int c = 0; c < C.n(); ++c) {
    L.off[c] = L.size;
    int r = 0;
    for (int s = 0; s < d; ++s)
      for (int b = 0; b < B.n(); ++b)
        if (B.q[b] - qp[s] == C.q[c]) {
          L.grp[c].push_back({b, s, r, B.dim[b]});
          r += B.dim[b];
        }
    L.rows[c] = r;
    L.size += (int64_t)r * C.dim[c];
  }
  return L;
}

// ------------------------------------------------------------------ task lists

void GemmList::add(GemmTask g) {
  if (g.M <= 0 || g.N <= 0) return;
  g.tiles_n = (g.N + tn - 1) / tn;
  g.tile0 = tiles;
  tiles += ((g.M + tm - 1) / tm) * g.tiles_n;
  t.push_back(g);
}

void GemmList::retile(int tm_, int tn_) {
  tm = tm_;
  tn = tn_;
  tiles = 0;
  for (auto& g : t) {
    g.tiles_n = (g.N + tn - 1) / tn;
    g.tile0 = tiles;
    tiles += ((g.M + tm - 1) / tm) * g.tiles_n;
  }
}

std::vector<GemmTask> GemmList::upload() {
  // Tasks in order of decreasing K (stable, so tasks of equal K keep their order and those sharing an operand stay
  // together): each XCD then starts its longest tiles first, and its last wave of workgroups holds the shortest.
  std::vector<GemmTask> out = t;
  std::stable_sort(out.begin(), out.end(), [](const GemmTask& a, const GemmTask& b) { return a.K > b.K; });
  int nt0 = 0;
  for (auto& g : out) {
    g.tile0 = nt0;
    nt0 += ((g.M + tm - 1) / tm) * g.tiles_n;
  }
  GemmTask rec{};
  int32_t s[kXcdRanges] = {};
  double total = 0.0;
  for (const auto& g : out) total += (double)((g.M + tm - 1) / tm) * g.tiles_n * (std::max(g.K, 0) + 64);
  // cut x at the first tile whose cumulative cost reaches x / 8 of the total
  int x = 1;
  double cum = 0.0;
  for (const auto& g : out) {
    const int nt = ((g.M + tm - 1) / tm) * g.tiles_n;
    const double c = std::max(g.K, 0) + 64;
    for (int i = 0; i < nt; ++i) {
      while (x < kXcdRanges - 1 && cum >= total * x / (kXcdRanges - 1)) s[x++] = g.tile0 + i;
      cum += c;
    }
  }
  while (x < kXcdRanges - 1) s[x++] = tiles;
  s[kXcdRanges - 1] = tiles;
  xmax = 0;
  for (int i = 0; i + 1 < kXcdRanges; ++i) xmax = std::max(xmax, s[i + 1] - s[i]);
  std::memcpy(&rec, s, sizeof(s));
  out.push_back(rec);
  return out;
}

double GemmList::efficiency(int tm_, int tn_) const {
  double use = 0, pad = 0;
  for (const auto& g : t) {
    const double k = std::max(g.K, 1);
    use += (double)g.M * g.N * k;
    pad += (double)((g.M + tm_ - 1) / tm_) * tm_ * ((g.N + tn_ - 1) / tn_) * tn_ * k;
  }
  return pad > 0 ? use / pad : 1.0;
}

void GemmList::choose_tile(bool allow_large) {
  int bm = 64, bn = 64;
  if (allow_large) {
    const double e0 = efficiency(64, 64);
    double best = 64 * 64 * e0;
    const int cand[3][2] = {{128, 64}, {64, 128}, {128, 128}};
    for (const auto& c : cand) {
      const double e = efficiency(c[0], c[1]);
      // a bigger tile halves operand traffic per flop; accept it unless padding eats that gain
      const double score = c[0] * c[1] * e;
      if (e >= 0.8 * e0 && score > best) {
        best = score;
        bm = c[0];
        bn = c[1];
      }
    }
  }
  retile(bm, bn);
}

double GemmList::flops() const {
  double f = 0;
  for (const auto& g : t) f += 2.0 * g.M * (double)g.N * g.K;
  return f;
}

void MixList::add(MixTask m, const std::vector<MixSrc>& s) {
  if (m.rows <= 0 || m.cols <= 0) return;
  m.src0 = (int)src.size();
  m.nsrc = (int)s.size();
  src.insert(src.end(), s.begin(), s.end());
  m.tiles_c = (m.cols + 63) / 64;
  m.tile0 = tiles;
  tiles += ((m.rows + 31) / 32) * m.tiles_c;
  t.push_back(m);
}

double MixList::flops() const {
  double f = 0;
  for (const auto& m : t) f += 2.0 * m.rows * (double)m.cols * m.nsrc;
  return f;
}

void ScaleList::add(ScaleTask s) {
  if (s.rows <= 0 || s.cols <= 0) return;
  s.tiles_c = (s.cols + 63) / 64;
  s.tile0 = tiles;
  tiles += ((s.rows + 31) / 32) * s.tiles_c;
  t.push_back(s);
}

int64_t frag_words(int R, int K) {
  return (int64_t)((R + kFragRows - 1) / kFragRows) * ((K + kFragK - 1) / kFragK) * kFragWords;
}

void PackList::add(PackTask p) {
  if (p.R <= 0 || p.nch <= 0) return;
  p.RB = (p.R + kFragRows - 1) / kFragRows;
  p.tile0 = tiles;
  tiles += (int)(((int64_t)p.RB * p.nch + 15) / 16);
  t.push_back(p);
}

// Pack of Z[R x K] into columns kc0 .. kc0 + 8 nch - 1 of a fragment matrix with KB k-fragments per row block.
static PackTask packtask(int prob, int R, int K, int sbase, int64_t soff, int ld, int trans, int dbase, int64_t doff,
                         int KB, int kc0, int nch) {
  PackTask p{};
  p.xbase = -1;
  p.shift_slot = -1;
  p.R = R; p.K = K; p.ld = ld; p.trans = trans;
  p.prob = prob; p.sbase = sbase; p.dbase = dbase;
  p.KB = KB; p.kc0 = kc0; p.nch = nch;
  p.soff = soff; p.doff = doff;
  return p;
}

static int kfrags(int K) { return (K + kFragK - 1) / kFragK; }
static int round8(int n) { return (n + 7) / 8 * 8; }
static int round4(int n) { return (n + 3) / 4 * 4; }

static GemmTask gemm(int prob, int M, int N, int K, int ab, int64_t ao, int lda, int bb, int64_t bo, int ldb, int cb,
                     int64_t co, int ldc, int beta) {
  GemmTask g{};
  g.M = M; g.N = N; g.K = K;
  g.lda = lda; g.ldb = ldb; g.ldc = ldc;
  g.prob = prob; g.beta = beta;
  g.abase = ab; g.bbase = bb; g.cbase = cb;
  g.aoff = ao; g.boff = bo; g.coff = co;
  return g;
}

static MixTask mixtask(int prob, int rows, int cols, int db, int64_t doff, int ldd) {
  MixTask m{};
  m.rows = rows; m.cols = cols; m.ldd = ldd; m.prob = prob; m.dbase = db; m.doff = doff;
  return m;
}

static MixSrc src(double coef, int base, int64_t off, int ld, int trans = 0) {
  MixSrc s{};
  s.coef = coef; s.base = base; s.off = off; s.ld = ld; s.trans = trans;
  return s;
}

// ------------------------------------------------------------------ H_eff

namespace {
struct W12Term { int w, u, t1, t2; double c; };

// sum_w' W1[w,w',s1,t1] W2[w',u,s2,t2], grouped by (s1, s2, u)
std::map<std::tuple<int, int, int>, std::vector<W12Term>> w12_terms(const Mpo& W1, const Mpo& W2) {
  std::map<std::tuple<int, int, int>, std::vector<W12Term>> out;
  const int d = W1.d;
  for (int w = 0; w < W1.dl; ++w)
    for (int u = 0; u < W2.dr; ++u)
      for (int s1 = 0; s1 < d; ++s1)
        for (int s2 = 0; s2 < d; ++s2)
          for (int t1 = 0; t1 < d; ++t1)
            for (int t2 = 0; t2 < d; ++t2) {
              double c = 0.0;
              for (int v = 0; v < W1.dr; ++v) c += W1.at(w, v, s1, t1) * W2.at(v, u, s2, t2);
              if (c != 0.0) out[std::make_tuple(s1, s2, u)].push_back({w, u, t1, t2, c});
            }
  return out;
}
}  // namespace

void build_heff(HeffPlan& p, int prob, const Leg& A, const Leg& B, const Mpo& W1, const Mpo& W2) {
  const std::vector<int>& qp = W1.qp;
  const PsiLayout X = psi_layout(A, B, qp);
  const EnvLLayout EL = envL_layout(A, W1.ql);
  const EnvRLayout ER = envR_layout(B, W2.qr);
  const int DL = W1.dl, DR = W2.dr;
  // T1: per psi block, [M_a' x db] (all non-identity L channels stacked)
  std::vector<int64_t> t1off(X.blk.size(), -1);
  int64_t nT1 = 0;
  for (size_t x = 0; x < X.blk.size(); ++x) {
    const auto& k = X.blk[x];
    if (EL.rows[k.a] == 0) continue;
    t1off[x] = nT1;
    nT1 += (int64_t)EL.rows[k.a] * k.db;
    p.g1.add(gemm(prob, EL.rows[k.a], k.db, k.da, 0, EL.stack_off[k.a], k.da, 2, k.off, k.db, 4, t1off[x], k.db, 0));
  }
  // T3: per right sector b, [rows_b x K_b]; row offset of each block inside it
  std::vector<int64_t> t3off(B.n(), 0);
  std::vector<int> rowin(X.blk.size(), 0);
  int64_t nT3 = 0;
  {
    std::vector<int> r(B.n(), 0);
    for (size_t x = 0; x < X.blk.size(); ++x) {
      rowin[x] = r[X.blk[x].b];
      r[X.blk[x].b] += X.blk[x].da;
    }
    for (int b = 0; b < B.n(); ++b) {
      t3off[b] = nT3;
      nT3 += (int64_t)X.b_rows[b] * ER.K[b];
    }
  }
  // Energy-shift structure of the low-precision copies (see plan.h): is L's
  // channel 0 exactly H_L and R's last channel exactly H_R?
  const int DM = W1.dr;
  auto only_identity = [](const Mpo& W, bool row, int idx, int keep) {
    const int n = row ? W.dr : W.dl;
    for (int v = 0; v < n; ++v)
      for (int s = 0; s < W.d; ++s)
        for (int t = 0; t < W.d; ++t) {
          const double w = row ? W.at(idx, v, s, t) : W.at(v, idx, s, t);
          if (w != ((v == keep && s == t) ? 1.0 : 0.0)) return false;
        }
    return true;
  };
  const bool shL = DL > 1 && W1.ql[0] == 0 && only_identity(W1, true, 0, 0) && only_identity(W2, true, 0, 0);
  const bool shR = DR > 1 && W2.qr[DR - 1] == 0 && only_identity(W2, false, DR - 1, DM - 1) &&
                   only_identity(W1, false, DM - 1, DL - 1);
  p.shiftL.push_back(shL ? 1 : 0);
  p.shiftR.push_back(shR ? 1 : 0);
  // Fragment form (split-bf16): L per column sector, x per block, T3 and R per right sector
  std::vector<int64_t> lf(A.n(), -1), xf(X.blk.size(), -1), t3f(B.n(), -1), rf(B.n(), -1);
  int64_t nLf = 0, nXf = 0, nT3f = 0, nRf = 0;
  for (int a = 0; a < A.n(); ++a) {
    if (EL.rows[a] == 0) continue;
    lf[a] = nLf;
    PackTask pt = packtask(prob, EL.rows[a], A.dim[a], 0, EL.stack_off[a], A.dim[a], 0, 0, nLf, kfrags(A.dim[a]), 0,
                           4 * kfrags(A.dim[a]));
    if (shL && EL.row_off[a][0] >= 0) {   // the H_L block of this column sector (a square diagonal block)
      pt.dr0 = EL.row_off[a][0];
      pt.dk0 = 0;
      pt.dlen = A.dim[a];
      pt.shift_slot = 2 * prob;
      DiagTask dg{};
      dg.prob = prob; dg.base = 0; dg.len = A.dim[a]; dg.ld = A.dim[a];
      dg.off = EL.stack_off[a] + (int64_t)EL.row_off[a][0] * A.dim[a];
      p.diagL.push_back(dg);
    }
    p.packL.add(pt);
    nLf += frag_words(EL.rows[a], A.dim[a]);
  }
  // x: every block is packed (the GEMM operand, where stage 1 uses it) and copied
  // to FP32 with rows padded to 4 (the mixing operand); T1 rows padded to 4
  std::vector<int64_t> t1f(X.blk.size(), -1), xm(X.blk.size(), -1);
  int64_t nT1f = 0, nXm = 0;
  for (size_t x = 0; x < X.blk.size(); ++x) {
    const auto& k = X.blk[x];
    xf[x] = nXf;   // B = x block [da x db], N-contiguous: fragment rows are its columns
    xm[x] = nXm;
    PackTask pt = packtask(prob, k.db, k.da, 2, k.off, k.db, 1, 2, nXf, kfrags(k.da), 0, 4 * kfrags(k.da));
    pt.xbase = 6;
    pt.xoff = nXm;
    pt.xld = round4(k.db);
    p.packX.add(pt);
    nXf += frag_words(k.db, k.da);
    nXm += (int64_t)k.da * round4(k.db);
    if (t1off[x] < 0) continue;
    t1f[x] = nT1f;
    nT1f += (int64_t)EL.rows[k.a] * round4(k.db);
    p.f1.add(gemm(prob, EL.rows[k.a], k.db, k.da, 0, lf[k.a], 0, 2, xf[x], 0, 4, t1f[x], round4(k.db), 0));
  }
  // K of T3 and R in the fragment form: channel u of right sector b starts at cpad[b][u], a multiple of 8
  std::vector<std::vector<int>> cpad(B.n());
  std::vector<int> Kp(B.n(), 0);
  for (int b = 0; b < B.n(); ++b) {
    cpad[b].assign(DR, -1);
    for (int u = 1; u < DR; ++u) {
      if (ER.col_off[b][u] < 0) continue;
      cpad[b][u] = Kp[b];
      Kp[b] += round8(B.dim[ER.b_in[b][u]]);
    }
  }
  for (int b = 0; b < B.n(); ++b) {
    if (ER.K[b] == 0 || X.b_rows[b] == 0) continue;
    const int KB = kfrags(Kp[b]);
    t3f[b] = nT3f;
    nT3f += frag_words(X.b_rows[b], Kp[b]);
    rf[b] = nRf;
    for (int u = 1; u < DR; ++u) {
      if (cpad[b][u] < 0) continue;
      const int du = B.dim[ER.b_in[b][u]];
      PackTask pt = packtask(prob, B.dim[b], du, 1, ER.off[b] + ER.col_off[b][u], ER.K[b], 0, 1, nRf, KB, cpad[b][u],
                             (du + 7) / 8);
      if (shR && u == DR - 1) {   // the H_R block of this row sector (b_in = b, square)
        pt.dr0 = 0;
        pt.dk0 = 0;
        pt.dlen = du;
        pt.shift_slot = 2 * prob + 1;
      }
      p.packR.add(pt);
    }
    // zeros past the last channel, to the end of the last k-fragment
    p.packR.add(packtask(prob, B.dim[b], 0, 1, 0, 0, 0, 1, nRf, KB, Kp[b], (KB * kFragK - Kp[b]) / 8));
    nRf += frag_words(B.dim[b], Kp[b]);
  }
  const auto terms = w12_terms(W1, W2);
  // Source of T1[w](a, t1, t2, b') = (L[w] x)(a, ...): psi block (a', t1, t2) with a' = a - ql[w]
  // (out: the FP64/FP32 form; outf: the fragment form with the padded T1 and x copies)
  auto source = [&](int a, int w, int t1, int t2, int bp, double c, std::vector<MixSrc>& out,
                    std::vector<MixSrc>& outf) {
    const int ap = A.find(A.q[a] - W1.ql[w]);
    if (ap < 0) return;
    const int xi = X.find(ap, t1, t2);
    if (xi < 0) return;
    const auto& k = X.blk[xi];
    if (k.b != bp) throw InvalidArg("internal: H_eff charge bookkeeping mismatch");
    if (w == DL - 1) {
      out.push_back(src(c, 6, k.off, k.db));
      outf.push_back(src(c, 6, xm[xi], round4(k.db)));
    } else {
      const int ro = EL.row_off[ap][w];
      if (ro < 0 || EL.a_out[ap][w] != a) return;
      out.push_back(src(c, 4, t1off[xi] + (int64_t)ro * k.db, k.db));
      outf.push_back(src(c, 4, t1f[xi] + (int64_t)ro * round4(k.db), round4(k.db)));
    }
  };
  for (size_t xo = 0; xo < X.blk.size(); ++xo) {
    const auto& ko = X.blk[xo];
    // R identity channel (u = 0): straight into y
    {
      std::vector<MixSrc> s, sf;
      auto it = terms.find(std::make_tuple(ko.s1, ko.s2, 0));
      if (it != terms.end())
        for (const auto& tm : it->second) source(ko.a, tm.w, tm.t1, tm.t2, ko.b, tm.c, s, sf);
      p.mixY.add(mixtask(prob, ko.da, ko.db, 3, ko.off, ko.db), s);
      p.mixYf.add(mixtask(prob, ko.da, ko.db, 3, ko.off, ko.db), sf);
    }
    for (int u = 1; u < DR; ++u) {
      const int co = ER.col_off[ko.b][u];
      if (co < 0) continue;
      const int bp = ER.b_in[ko.b][u];
      std::vector<MixSrc> s, sf;
      auto it = terms.find(std::make_tuple(ko.s1, ko.s2, u));
      if (it != terms.end())
        for (const auto& tm : it->second) source(ko.a, tm.w, tm.t1, tm.t2, bp, tm.c, s, sf);
      p.mixT.add(mixtask(prob, ko.da, B.dim[bp], 5, t3off[ko.b] + (int64_t)rowin[xo] * ER.K[ko.b] + co, ER.K[ko.b]),
                 s);
      MixTask mf = mixtask(prob, ko.da, B.dim[bp], 5, t3f[ko.b], kfrags(Kp[ko.b]));
      mf.r0 = rowin[xo];
      mf.c0 = cpad[ko.b][u];
      p.mixTf.add(mf, sf);
    }
  }
  if (shR)
    for (int b = 0; b < B.n(); ++b) {
      const int co = ER.col_off[b][DR - 1];
      if (co < 0) continue;
      DiagTask dg{};
      dg.prob = prob; dg.base = 1; dg.len = B.dim[b]; dg.ld = ER.K[b];
      dg.off = ER.off[b] + co;
      p.diagR.push_back(dg);
    }
  for (int b = 0; b < B.n(); ++b) {
    if (ER.K[b] == 0 || X.b_rows[b] == 0) continue;
    p.g2.add(gemm(prob, X.b_rows[b], B.dim[b], ER.K[b], 5, t3off[b], ER.K[b], 1, ER.off[b], ER.K[b], 3,
                  X.b_first[b], B.dim[b], 1));
    p.f2.add(gemm(prob, X.b_rows[b], B.dim[b], Kp[b], 5, t3f[b], 0, 1, rf[b], 0, 3, X.b_first[b], B.dim[b], 1));
  }
  p.n_psi.push_back(X.size);
  p.n_Lf.push_back(nLf);
  p.n_Rf.push_back(nRf);
  p.n_Xf.push_back(nXf);
  p.n_T3f.push_back(nT3f);
  p.n_T1f.push_back(nT1f);
  p.n_Xm.push_back(nXm);
  p.n_T1.push_back(nT1);
  p.n_T3.push_back(nT3);
  p.n_L.push_back(EL.size);
  p.n_R.push_back(ER.size);
}

static void in_bounds(int64_t lo, int64_t hi, const std::vector<int64_t>& sizes, int prob, int base,
                      const char* what) {
  const size_t k = (size_t)prob * kNumBases + base;
  if (base < 0 || base >= kNumBases || k >= sizes.size() || sizes[k] < 0 || lo < 0 || hi >= sizes[k])
    throw InvalidArg(std::string("internal: ") + what + " plan touches memory outside its buffer");
}

void check_gemm(const GemmList& g, int mode, const std::vector<int64_t>& sizes, const char* what) {
  for (const auto& t : g.t) {
    if (t.M <= 0 || t.N <= 0) continue;
    in_bounds(t.coff, t.coff + (int64_t)(t.M - 1) * t.ldc + t.N - 1, sizes, t.prob, t.cbase, what);
    if (t.ldc < t.N) throw InvalidArg(std::string("internal: ") + what + " ldc < N");
    if (t.K <= 0) continue;
    const int64_t a_hi = mode == 2 ? t.aoff + (int64_t)(t.K - 1) * t.lda + t.M - 1
                                   : t.aoff + (int64_t)(t.M - 1) * t.lda + t.K - 1;
    const int64_t b_hi = mode == 1 ? t.boff + (int64_t)(t.N - 1) * t.ldb + t.K - 1
                                   : t.boff + (int64_t)(t.K - 1) * t.ldb + t.N - 1;
    in_bounds(t.aoff, a_hi, sizes, t.prob, t.abase, what);
    in_bounds(t.boff, b_hi, sizes, t.prob, t.bbase, what);
    // the kernels address operands by 32-bit offsets from the task's base
    if (a_hi - t.aoff >= INT32_MAX || b_hi - t.boff >= INT32_MAX)
      throw InvalidArg(std::string(what) + ": one GEMM operand spans 2^31 elements or more");
  }
}

std::vector<int> fused_qp(const std::vector<int>& qp) {
  const int d = (int)qp.size();
  std::vector<int> f((size_t)d * d);
  for (int s1 = 0; s1 < d; ++s1)
    for (int s2 = 0; s2 < d; ++s2) f[(size_t)s1 * d + s2] = qp[s1] + qp[s2];
  return f;
}

void build_twosite_V(MixList& m, int prob, const Leg& A, const Leg& B, const std::vector<int>& qp) {
  const int d = (int)qp.size();
  const PsiLayout P = psi_layout(A, B, qp);
  const IsoLayout V = V_layout(B, fused_qp(qp), A);
  for (const auto& k : P.blk) {
    const int r = V.row_of(k.a, k.b, k.s1 * d + k.s2);
    if (r < 0) throw InvalidArg("internal: a two-site block has no rows in the fused V layout");
    MixTask t{};
    t.rows = k.db;                // rows of V: the right sector's states
    t.cols = k.da;                // columns of V: the left sector's states
    t.ldd = A.dim[k.a];
    t.prob = prob;
    t.dbase = 1;
    t.doff = V.off[k.a] + (int64_t)r * A.dim[k.a];
    MixSrc src{};
    src.coef = 1.0;
    src.off = k.off;
    src.ld = k.db;
    src.base = 0;
    src.trans = 1;                // V(r, c) = psi block (c, r)
    m.add(t, {src});
  }
}

void build_overlap(std::vector<OverlapSeg>& segs, int item, const Leg& leg, const std::vector<int>& ql,
                   const std::vector<int>& qr, int wl, int wr) {
  if (wl < 0 || wl >= (int)ql.size() - 1 || wr < 1 || wr >= (int)qr.size())
    throw InvalidArg("overlap: channel out of range");
  if (ql[wl] != qr[wr]) throw InvalidArg("overlap: the two channels carry different charges");
  const EnvLLayout L = envL_layout(leg, ql);
  const EnvRLayout R = envR_layout(leg, qr);
  for (int ac = 0; ac < leg.n(); ++ac) {
    if (L.row_off[ac][wl] < 0) continue;
    const int ar = L.a_out[ac][wl];
    if (R.col_off[ar][wr] < 0 || R.b_in[ar][wr] != ac) throw InvalidArg("internal: overlap blocks do not match");
    OverlapSeg g{};
    g.item = item;
    g.rows = leg.dim[ar];
    g.cols = leg.dim[ac];
    g.aoff = L.stack_off[ac] + (int64_t)L.row_off[ac][wl] * leg.dim[ac];
    g.lda = leg.dim[ac];
    g.boff = R.off[ar] + R.col_off[ar][wr];
    g.ldb = R.K[ar];
    segs.push_back(g);
  }
}

void check_mix(const MixList& m, const std::vector<int64_t>& sizes, const char* what) {
  for (const auto& t : m.t) {
    if (t.rows <= 0 || t.cols <= 0) continue;
    in_bounds(t.doff, t.doff + (int64_t)(t.rows - 1) * t.ldd + t.cols - 1, sizes, t.prob, t.dbase, what);
    for (int k = 0; k < t.nsrc; ++k) {
      const MixSrc& s = m.src[t.src0 + k];
      const int64_t hi = s.trans ? s.off + (int64_t)(t.cols - 1) * s.ld + t.rows - 1
                                 : s.off + (int64_t)(t.rows - 1) * s.ld + t.cols - 1;
      in_bounds(s.off, hi, sizes, t.prob, s.base, what);
    }
  }
}

// Last word of a fragment-layout matrix [R x K] at off, and a check that its
// byte extent fits the kernels' 32-bit offsets.
static int64_t frag_last(int64_t off, int R, int K, const char* what) {
  const int64_t w = frag_words(R, K);
  if (w * 4 >= INT32_MAX) throw InvalidArg(std::string(what) + ": one fragment-layout operand spans 2 GiB or more");
  return off + w - 1;
}

void check_gemm_frag(const GemmList& g, const std::vector<int64_t>& sizes, const char* what) {
  for (const auto& t : g.t) {
    if (t.M <= 0 || t.N <= 0) continue;
    in_bounds(t.coff, t.coff + (int64_t)(t.M - 1) * t.ldc + t.N - 1, sizes, t.prob, t.cbase, what);
    if (t.ldc < t.N) throw InvalidArg(std::string("internal: ") + what + " ldc < N");
    if (t.K <= 0) continue;
    in_bounds(t.aoff, frag_last(t.aoff, t.M, t.K, what), sizes, t.prob, t.abase, what);
    in_bounds(t.boff, frag_last(t.boff, t.N, t.K, what), sizes, t.prob, t.bbase, what);
  }
}

void check_mix_frag(const MixList& m, const std::vector<int64_t>& sizes, const char* what) {
  for (const auto& t : m.t) {
    if (t.rows <= 0 || t.cols <= 0) continue;
    // the destination is a fragment matrix with ldd k-fragments per row block; the
    // task writes rows [r0, r0 + rows) and columns [c0, c0 + round8(cols)) of it
    if (t.r0 < 0 || t.c0 < 0 || t.c0 % 8 != 0 || t.c0 + round8(t.cols) > t.ldd * kFragK)
      throw InvalidArg(std::string("internal: ") + what + " fragment block outside its matrix");
    const int64_t last = t.doff + ((int64_t)((t.r0 + t.rows - 1) / kFragRows) * t.ldd + t.ldd) * kFragWords - 1;
    in_bounds(t.doff, last, sizes, t.prob, t.dbase, what);
    for (int k = 0; k < t.nsrc; ++k) {
      const MixSrc& s = m.src[t.src0 + k];
      const int64_t hi = s.trans ? s.off + (int64_t)(t.cols - 1) * s.ld + t.rows - 1
                                 : s.off + (int64_t)(t.rows - 1) * s.ld + t.cols - 1;
      in_bounds(s.off, hi, sizes, t.prob, s.base, what);
    }
  }
}

void check_mix_v4(const MixList& m, const std::vector<int64_t>& sizes, const char* what) {
  for (const auto& t : m.t) {
    if (t.rows <= 0 || t.cols <= 0) continue;
    for (int k = 0; k < t.nsrc; ++k) {
      const MixSrc& s = m.src[t.src0 + k];
      if (s.trans) continue;
      if (s.off % 4 != 0 || s.ld % 4 != 0 || s.ld < round4(t.cols))
        throw InvalidArg(std::string("internal: ") + what + " source rows not 16-byte aligned and padded");
      in_bounds(s.off, s.off + (int64_t)(t.rows - 1) * s.ld + round4(t.cols) - 1, sizes, t.prob, s.base, what);
    }
  }
}

void check_pack(const PackList& pl, const std::vector<int64_t>& ssizes, const std::vector<int64_t>& dsizes,
                const char* what) {
  for (const auto& t : pl.t) {
    if (t.K > 0) {
      const int64_t hi = t.trans ? t.soff + (int64_t)(t.K - 1) * t.ld + t.R - 1
                                 : t.soff + (int64_t)(t.R - 1) * t.ld + t.K - 1;
      in_bounds(t.soff, hi, ssizes, t.prob, t.sbase, what);
    }
    if (t.kc0 < 0 || t.kc0 % 8 != 0 || t.K > 8 * t.nch || t.kc0 + 8 * t.nch > t.KB * kFragK)
      throw InvalidArg(std::string("internal: ") + what + " pack outside its fragment matrix");
    if (t.xbase >= 0 && t.K > 0) {   // FP32 copy, in the source's orientation
      const int rows = t.trans ? t.K : t.R, cols = t.trans ? t.R : t.K;
      if (t.xld < cols) throw InvalidArg(std::string("internal: ") + what + " copy row shorter than the block");
      in_bounds(t.xoff, t.xoff + (int64_t)(rows - 1) * t.xld + cols - 1, dsizes, t.prob, t.xbase, what);
    }
    in_bounds(t.doff, frag_last(t.doff, t.R, t.KB * kFragK, what), dsizes, t.prob, t.dbase, what);
  }
}

void check_scale(const ScaleList& sl, const std::vector<int64_t>& sizes, const char* what, int64_t colmap_bound) {
  for (const auto& t : sl.t) {
    if (t.rows <= 0 || t.cols <= 0) continue;
    in_bounds(t.doff, t.doff + (int64_t)(t.rows - 1) * t.ldd + t.cols - 1, sizes, t.prob, t.dbase, what);
    const int64_t scol = t.colmap >= 0 ? t.lds - 1 : t.cols - 1;
    if (t.colmap >= 0 && (t.colmap < 0 || t.colmap + t.cols > colmap_bound))
      throw InvalidArg(std::string("internal: ") + what + " column map out of range");
    in_bounds(t.soff, t.soff + (int64_t)(t.rows - 1) * t.lds + scol, sizes, t.prob, t.sbase, what);
    if (t.rbase >= 0) in_bounds(t.roff, t.roff + t.rows - 1, sizes, t.prob, t.rbase, what);
    if (t.cbase >= 0) in_bounds(t.coff, t.coff + t.cols - 1, sizes, t.prob, t.cbase, what);
  }
}

void heff_work(const Leg& A, const Leg& B, const Mpo& W1, const Mpo& W2, double& flops, double& bytes) {
  HeffPlan p;
  build_heff(p, 0, A, B, W1, W2);
  flops = p.g1.flops() + p.g2.flops() + p.mixY.flops() + p.mixT.flops();
  bytes = 8.0 * (double)(p.n_L[0] + p.n_R[0] + 2 * p.n_psi[0]);
}

// ------------------------------------------------------------------ environments

void build_envL(EnvPlan& p, int prob, const Leg& A, const Leg& C, const Mpo& W) {
  const std::vector<int>& qp = W.qp;
  const EnvLLayout EL = envL_layout(A, W.ql);
  const EnvLLayout EN = envL_layout(C, W.qr);
  const IsoLayout U = U_layout(A, qp, C);
  const int DL = W.dl, DM = W.dr;
  // T_a[(c', a', s')] = Lstack_{a'} @ U_{c'}[(a', s') rows]   [M_a' x k_c']
  std::map<std::tuple<int, int, int>, int64_t> taoff;
  int64_t nTa = 0;
  for (int cp = 0; cp < C.n(); ++cp)
    for (const auto& g : U.grp[cp]) {
      const int ap = g.sec;
      if (EL.rows[ap] == 0) continue;
      taoff[std::make_tuple(cp, ap, g.s)] = nTa;
      p.ga.add(gemm(prob, EL.rows[ap], C.dim[cp], A.dim[ap], 0, EL.stack_off[ap], A.dim[ap], 1,
                    U.off[cp] + (int64_t)g.row * C.dim[cp], C.dim[cp], 3, nTa, C.dim[cp], 0));
      nTa += (int64_t)EL.rows[ap] * C.dim[cp];
    }
  // T_2[w', c'] = [r_c x k_c'] in U_c row order, c = c' + qr[w']
  int64_t nT2 = 0;
  for (int w2 = 0; w2 < DM - 1; ++w2)
    for (int cp = 0; cp < C.n(); ++cp) {
      const int c = C.find(C.q[cp] + W.qr[w2]);
      if (c < 0) continue;
      const int64_t base = nT2;
      nT2 += (int64_t)U.rows[c] * C.dim[cp];
      for (const auto& g : U.grp[c]) {   // row group (a, s) of U_c
        const int a = g.sec, s = g.s;
        std::vector<MixSrc> ss;
        for (int w = 0; w < DL; ++w)
          for (int sp = 0; sp < W.d; ++sp) {
            const double cf = W.at(w, w2, s, sp);
            if (cf == 0.0) continue;
            const int ap = A.find(A.q[a] - W.ql[w]);
            if (ap < 0) continue;
            const int urow = U.row_of(cp, ap, sp);
            if (urow < 0) continue;
            if (w == DL - 1) {
              ss.push_back(src(cf, 1, U.off[cp] + (int64_t)urow * C.dim[cp], C.dim[cp]));
            } else {
              const int ro = EL.row_off[ap][w];
              if (ro < 0) continue;
              ss.push_back(src(cf, 3, taoff.at(std::make_tuple(cp, ap, sp)) + (int64_t)ro * C.dim[cp], C.dim[cp]));
            }
          }
        p.mix.add(mixtask(prob, g.dim, C.dim[cp], 4, base + (int64_t)g.row * C.dim[cp], C.dim[cp]), ss);
      }
      // L'[w'](c, c') = U_c^T T_2    (TN)
      p.gc.add(gemm(prob, C.dim[c], C.dim[cp], U.rows[c], 1, U.off[c], C.dim[c], 4, base, C.dim[cp], 2,
                    EN.stack_off[cp] + (int64_t)EN.row_off[cp][w2] * C.dim[cp], C.dim[cp], 0));
    }
  p.n_T1.push_back(nTa);
  p.n_T2.push_back(nT2);
  p.n_new.push_back(EN.size);
}

void build_envR(EnvPlan& p, int prob, const Leg& B, const Leg& C, const Mpo& W) {
  const std::vector<int>& qp = W.qp;
  const EnvRLayout ER = envR_layout(B, W.qr);
  const EnvRLayout EN = envR_layout(C, W.ql);
  const IsoLayout V = V_layout(B, qp, C);
  const int DM = W.dl, DR = W.dr;
  // P[(c, s, b)] = V_c[(s, b) rows]^T @ R_b   [k_c x K_b]   (TN)
  std::map<std::tuple<int, int, int>, int64_t> poff;
  int64_t nP = 0;
  for (int c = 0; c < C.n(); ++c)
    for (const auto& g : V.grp[c]) {
      const int b = g.sec;
      if (ER.K[b] == 0) continue;
      poff[std::make_tuple(c, g.s, b)] = nP;
      p.ga.add(gemm(prob, C.dim[c], ER.K[b], B.dim[b], 1, V.off[c] + (int64_t)g.row * C.dim[c], C.dim[c], 0,
                    ER.off[b], ER.K[b], 3, nP, ER.K[b], 0));
      nP += (int64_t)C.dim[c] * ER.K[b];
    }
  // Q[w, c] = [k_c x r'_c'] with columns in V_c' row order, c' = c - ql[w]
  int64_t nQ = 0;
  for (int w = 1; w < DM; ++w)
    for (int c = 0; c < C.n(); ++c) {
      const int cp = C.find(C.q[c] - W.ql[w]);
      if (cp < 0) continue;
      const int64_t base = nQ;
      nQ += (int64_t)C.dim[c] * V.rows[cp];
      for (const auto& g : V.grp[cp]) {   // column group (s', b') of V_c'
        const int bp = g.sec, sp = g.s;
        std::vector<MixSrc> ss;
        for (int u = 0; u < DR; ++u)
          for (int s = 0; s < W.d; ++s) {
            const double cf = W.at(w, u, s, sp);
            if (cf == 0.0) continue;
            const int b = B.find(C.q[c] + qp[s]);
            if (b < 0) continue;
            const int vrow = V.row_of(c, b, s);
            if (vrow < 0) continue;
            if (u == 0) {
              if (b != bp) continue;
              ss.push_back(src(cf, 1, V.off[c] + (int64_t)vrow * C.dim[c], C.dim[c], 1));
            } else {
              const int co = ER.col_off[b][u];
              if (co < 0 || ER.b_in[b][u] != bp) continue;
              ss.push_back(src(cf, 3, poff.at(std::make_tuple(c, s, b)) + co, ER.K[b]));
            }
          }
        p.mix.add(mixtask(prob, C.dim[c], g.dim, 4, base + g.row, V.rows[cp]), ss);
      }
      // R'[w](c, c') = Q V_c'   (NN)
      p.gc.add(gemm(prob, C.dim[c], C.dim[cp], V.rows[cp], 4, base, V.rows[cp], 1, V.off[cp], C.dim[cp], 2,
                    EN.off[c] + EN.col_off[c][w], EN.K[c], 0));
    }
  p.n_T1.push_back(nP);
  p.n_T2.push_back(nQ);
  p.n_new.push_back(EN.size);
}

// ------------------------------------------------------------------ prediction

void build_predict(PredictPlan& p, int prob, const Leg& Aa, const Leg& Bt, const Leg& Bb, const std::vector<int>& qp) {
  const IsoLayout V = V_layout(Bt, qp, Aa);     // V_i: rows (s, beta), columns alpha
  const IsoLayout U = U_layout(Bt, qp, Bb);     // U_{i+1}: rows (beta, s'), columns alpha'
  const PsiLayout X = psi_layout(Aa, Bb, qp);
  // lambda offsets
  std::vector<int64_t> la(Aa.n()), lt(Bt.n()), lb(Bb.n());
  {
    int64_t o = 0;
    for (int k = 0; k < Aa.n(); ++k) { la[k] = o; o += Aa.dim[k]; }
    o = 0;
    for (int k = 0; k < Bt.n(); ++k) { lt[k] = o; o += Bt.dim[k]; }
    o = 0;
    for (int k = 0; k < Bb.n(); ++k) { lb[k] = o; o += Bb.dim[k]; }
  }
  // V scaled: columns by lam_i
  for (int c = 0; c < Aa.n(); ++c) {
    ScaleTask s{};
    s.rows = V.rows[c]; s.cols = Aa.dim[c]; s.lds = Aa.dim[c]; s.ldd = Aa.dim[c];
    s.prob = prob; s.sbase = 1; s.dbase = 6; s.rbase = -1; s.cbase = 0; s.invert_row = 0; s.colmap = -1;
    s.soff = V.off[c]; s.doff = V.off[c]; s.coff = la[c];
    p.scale.add(s);
  }
  // U scaled: rows by 1/lam_prev (floored), columns by lam_ip1
  for (int c = 0; c < Bb.n(); ++c)
    for (const auto& g : U.grp[c]) {
      ScaleTask s{};
      s.rows = g.dim; s.cols = Bb.dim[c]; s.lds = Bb.dim[c]; s.ldd = Bb.dim[c];
      s.prob = prob; s.sbase = 3; s.dbase = 7; s.rbase = 2; s.cbase = 4; s.invert_row = 1; s.colmap = -1;
      s.soff = U.off[c] + (int64_t)g.row * Bb.dim[c]; s.doff = s.soff; s.roff = lt[g.sec]; s.coff = lb[c];
      p.scale.add(s);
    }
  for (const auto& k : X.blk) {
    const int bt = Bt.find(Aa.q[k.a] + qp[k.s1]);
    int vrow = -1, urow = -1;
    if (bt >= 0) {
      vrow = V.row_of(k.a, bt, k.s1);
      urow = U.row_of(k.b, bt, k.s2);
    }
    if (bt < 0 || vrow < 0 || urow < 0) {
      p.g.add(gemm(prob, k.da, k.db, 0, 6, 0, 1, 7, 0, 1, 5, k.off, k.db, 0));   // zero block
      continue;
    }
    p.g.add(gemm(prob, k.da, k.db, Bt.dim[bt], 6, V.off[k.a] + (int64_t)vrow * Aa.dim[k.a], Aa.dim[k.a], 7,
                 U.off[k.b] + (int64_t)urow * Bb.dim[k.b], Bb.dim[k.b], 5, k.off, k.db, 0));
  }
  p.n_Vs.push_back(V.size);
  p.n_Us.push_back(U.size);
}

}  // namespace idmrg
