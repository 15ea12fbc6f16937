// TEST INFRASTRUCTURE ONLY.
//
// Oracle of the learned multipole-acceptance criterion layered on the group
// walk of Sec. 2.2 (the paper itself has only the opening angle theta).
// Plain FP64 with the BF16 rounding points of the GPU network mirrored.
// Definitions fixed here (readings of the target's description):
//   * Band: a candidate the opening test accepts at theta_lo is accepted; one
//     it opens at theta_hi is opened; in between the network decides.
//   * 12 features of (group g, cell c), computed in FP32 from the FP32 tree
//     (see mac_features below).
//   * Label: e = max over the group's particles i of
//     |a_pc(i; c) - sum_{j in c} a_pp(i, j)| / |a_i(direct)|, target
//     y = log10(max(e, 1e-12)).
//   * Network 12-64-64-1 with ReLU: inputs, weights and hidden activations
//     rounded to BF16 (round to nearest even) before each product, sums in
//     FP64 here (FP32 on the GPU); pinball loss at quantile tau; Adam with
//     bias correction.
//   * Decision: accept iff yhat <= log10(tau_pair).  If the root of the sum
//     over a group's network-accepted candidates of 10^(2 yhat) exceeds the
//     budget, the group's lists are those of the plain theta walk instead
//     (a negative budget sends every group back to theta).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <vector>

#include <omp.h>

#include "oracle_tree.h"

namespace orc {
namespace {

constexpr int kIn = 12, kH = 64;
constexpr int oW1 = 0, oB1 = oW1 + kH * kIn, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH,
              oB3 = oW3 + kH, kParams = oB3 + 1;  // 5057

// Round to BF16 (nearest even) through FP32, returned as a double.
double bf16(double v) {
  float f = (float)v;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  u &= 0xFFFF0000u;
  std::memcpy(&f, &u, 4);
  return (double)f;
}

// The 12 features of candidate cell c for the group whose cell is gc.
void mac_features(const Tree& t, int32_t gc, int32_t c, float* f) {
  float gmin[3], gmax[3];
  group_box(t, gc, gmin, gmax);
  const Cell& cc = t.cells[c];
  const float* geo = cc.geo;
  const float l = geo[3];
  float tt[3];
  for (int k = 0; k < 3; ++k) {
    float a = gmin[k] - geo[k], b = geo[k] - gmax[k];
    float m = a > b ? a : b;
    tt[k] = m > 0.0f ? m : 0.0f;
  }
  const float d2 = (tt[0] * tt[0] + tt[1] * tt[1]) + tt[2] * tt[2];
  const float d = std::sqrt(d2);
  const float Mc = (float)cc.M, Mtot = (float)t.cells[0].M;
  float q[6];
  for (int k = 0; k < 6; ++k) q[k] = (float)cc.Q[k];
  const float qn = std::sqrt((q[0] * q[0] + q[1] * q[1] + q[2] * q[2]) +
                             2.0f * (q[3] * q[3] + q[4] * q[4] + q[5] * q[5]));
  float ge[3];
  for (int k = 0; k < 3; ++k) ge[k] = gmax[k] - gmin[k];
  const float rg = 0.5f * std::sqrt((ge[0] * ge[0] + ge[1] * ge[1]) + ge[2] * ge[2]);
  f[0] = d / l;
  f[1] = std::log10(Mc / Mtot) / 3.0f;
  f[2] = qn / (Mc * l * l);
  f[3] = std::log2(1.0f + rg / l);
  for (int k = 0; k < 3; ++k) f[4 + k] = (float)(cc.mx[k] - cc.mn[k]) / l;
  for (int k = 0; k < 3; ++k) f[7 + k] = std::log2(1.0f + ge[k] / l);
  f[10] = std::log2(1.0f + (float)cc.depth) / std::log2(22.0f);
  float s = 0.0f;
  for (int k = 0; k < 3; ++k) {
    const float dc = (float)cc.com[k] - geo[k];
    s += dc * dc;
  }
  f[11] = std::sqrt(s) / l;
}

// One sample through the network; keeps what the backward pass needs.
struct Fwd {
  double x[kIn], a1[kH], h1[kH], a2[kH], h2[kH], y;
};

void forward(const double* P, const float* xin, bool rnd, Fwd& s) {
  auto R = [&](double v) { return rnd ? bf16(v) : v; };
  for (int k = 0; k < kIn; ++k) s.x[k] = R(xin[k]);
  for (int j = 0; j < kH; ++j) {
    double a = 0;
    for (int k = 0; k < kIn; ++k) a += R(P[oW1 + j * kIn + k]) * s.x[k];
    s.a1[j] = a + P[oB1 + j];
    s.h1[j] = R(std::max(0.0, s.a1[j]));
  }
  for (int j = 0; j < kH; ++j) {
    double a = 0;
    for (int k = 0; k < kH; ++k) a += R(P[oW2 + j * kH + k]) * s.h1[k];
    s.a2[j] = a + P[oB2 + j];
    s.h2[j] = R(std::max(0.0, s.a2[j]));
  }
  double y = 0;
  for (int k = 0; k < kH; ++k) y += R(P[oW3 + k]) * s.h2[k];
  s.y = y + P[oB3];
}

// Walk of one group with the learned criterion; `score` gives yhat for a
// band candidate.  Returns true if the group fell back to the theta walk.
template <typename Score>
bool walk_learned(const Tree& t, int32_t gc, float theta, float th_lo, float th_hi, float log10_tau,
                  float budget, Score score, std::vector<int32_t>& C, std::vector<int32_t>& Lv) {
  C.clear();
  Lv.clear();
  if (t.cells[0].n_child == 0) {
    Lv.push_back(0);
    return false;
  }
  float gmin[3], gmax[3];
  group_box(t, gc, gmin, gmax);
  const float lo2 = th_lo * th_lo, hi2 = th_hi * th_hi;
  double sum2 = 0;
  std::vector<int32_t> stack{0};
  while (!stack.empty()) {
    const Cell& nc = t.cells[stack.back()];
    stack.pop_back();
    for (int k = 0; k < nc.n_child; ++k) {
      const int32_t c = nc.first_child + k;
      const float* geo = t.cells[c].geo;
      bool open;
      if (!mac_open(gmin, gmax, geo, lo2)) {
        open = false;  // hard accept
      } else if (mac_open(gmin, gmax, geo, hi2)) {
        open = true;  // hard open
      } else {
        const float yh = score(c);
        open = !(yh <= log10_tau);
        if (!open) sum2 += std::pow(10.0, 2.0 * (double)yh);
      }
      if (open) {
        if (t.cells[c].n_child == 0) Lv.push_back(c);
        else stack.push_back(c);
      } else {
        C.push_back(c);
      }
    }
  }
  if (std::sqrt(sum2) > (double)budget) {
    walk_group(t, gc, theta, C, Lv);
    return true;
  }
  std::sort(C.begin(), C.end());
  std::sort(Lv.begin(), Lv.end());
  return false;
}

}  // namespace
}  // namespace orc

using namespace orc;

extern "C" {

int orc_mlp_params(void) { return kParams; }

// Features of n (group index, cell id) pairs: out[n x 12].
int orc_mac_features(const void* h, const int32_t* g, const int32_t* c, int64_t n, float* out) {
  const Tree& t = *(const Tree*)h;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) mac_features(t, t.groups[g[i]], c[i], out + kIn * i);
  return 0;
}

// Band candidates of theta_lo walks of the selected groups (all if sel ==
// NULL): candidates the theta_lo test opens and the theta_hi test does not.
// Appends (group index, cell id) in walk order (groups ascending, cells
// ascending within a group); *n_out = total (pairs beyond cap not written).
int orc_mac_band(const void* h, float th_lo, float th_hi, const int32_t* sel, int64_t nsel,
                 int32_t* g_out, int32_t* c_out, int64_t cap, int64_t* n_out) {
  const Tree& t = *(const Tree*)h;
  const int64_t ng = sel ? nsel : (int64_t)t.groups.size();
  const float lo2 = th_lo * th_lo, hi2 = th_hi * th_hi;
  std::vector<std::vector<int32_t>> band(ng);
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t u = 0; u < ng; ++u) {
    const int32_t gi = sel ? sel[u] : (int32_t)u, gc = t.groups[gi];
    if (t.cells[0].n_child == 0) continue;
    float gmin[3], gmax[3];
    group_box(t, gc, gmin, gmax);
    std::vector<int32_t> stack{0};
    while (!stack.empty()) {
      const Cell& nc = t.cells[stack.back()];
      stack.pop_back();
      for (int k = 0; k < nc.n_child; ++k) {
        const int32_t c = nc.first_child + k;
        if (!mac_open(gmin, gmax, t.cells[c].geo, lo2)) continue;
        if (!mac_open(gmin, gmax, t.cells[c].geo, hi2)) band[u].push_back(c);
        if (t.cells[c].n_child) stack.push_back(c);
      }
    }
    std::sort(band[u].begin(), band[u].end());
  }
  int64_t k = 0;
  for (int64_t u = 0; u < ng; ++u)
    for (int32_t c : band[u]) {
      if (k < cap) {
        g_out[k] = sel ? sel[u] : (int32_t)u;
        c_out[k] = c;
      }
      ++k;
    }
  *n_out = k;
  return 0;
}

// Labels e(g, c) in FP64; acc_direct [n x 3] by input index.
int orc_mac_labels(const void* h, const double* acc_direct, float eps, const int32_t* g,
                   const int32_t* c, int64_t n, double* e_out) {
  const Tree& t = *(const Tree*)h;
  const double eps2 = (double)eps * (double)eps;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t u = 0; u < n; ++u) {
    const Cell& gcell = t.cells[t.groups[g[u]]];
    const Cell& cc = t.cells[c[u]];
    double emax = 0;
    for (int64_t ii = gcell.first; ii < gcell.first + gcell.n; ++ii) {
      const int32_t i = t.order[ii];
      const double xi = t.x[0][i], yi = t.x[1][i], zi = t.x[2][i];
      // the cell's multipole at x_i
      const double R0 = xi - cc.com[0], R1 = yi - cc.com[1], R2 = zi - cc.com[2];
      const double r2 = R0 * R0 + R1 * R1 + R2 * R2 + eps2;
      const double ri = 1.0 / std::sqrt(r2), ri2 = ri * ri, ri3 = ri * ri2, ri5 = ri3 * ri2,
                   ri7 = ri5 * ri2;
      const double* Q = cc.Q;
      const double q0 = Q[0] * R0 + Q[3] * R1 + Q[4] * R2;
      const double q1 = Q[3] * R0 + Q[1] * R1 + Q[5] * R2;
      const double q2 = Q[4] * R0 + Q[5] * R1 + Q[2] * R2;
      const double s = R0 * q0 + R1 * q1 + R2 * q2;
      double ap[3] = {-cc.M * R0 * ri3 + q0 * ri5 - 2.5 * s * R0 * ri7,
                      -cc.M * R1 * ri3 + q1 * ri5 - 2.5 * s * R1 * ri7,
                      -cc.M * R2 * ri3 + q2 * ri5 - 2.5 * s * R2 * ri7};
      // the exact sum over the cell's particles
      double ax = 0, ay = 0, az = 0;
      for (int64_t jj = cc.first; jj < cc.first + cc.n; ++jj) {
        const int32_t j = t.order[jj];
        if (j == i) continue;
        const double D0 = t.x[0][j] - xi, D1 = t.x[1][j] - yi, D2 = t.x[2][j] - zi;
        const double d2 = D0 * D0 + D1 * D1 + D2 * D2 + eps2;
        const double w = t.m[j] / (d2 * std::sqrt(d2));
        ax += w * D0;
        ay += w * D1;
        az += w * D2;
      }
      const double dx = ap[0] - ax, dy = ap[1] - ay, dz = ap[2] - az;
      const double* ad = acc_direct + 3 * i;
      const double na = std::sqrt(ad[0] * ad[0] + ad[1] * ad[1] + ad[2] * ad[2]);
      emax = std::max(emax, std::sqrt(dx * dx + dy * dy + dz * dz) / na);
    }
    e_out[u] = emax;
  }
  return 0;
}

// Forward pass of B samples x [B x 12]; P = 5057 parameters (W1 [64x12],
// b1, W2 [64x64], b2, w3 [64], b3).  round_bf16 != 0 mirrors the GPU.
int orc_mlp_forward(const double* P, const float* x, int64_t B, int round_bf16, double* y) {
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < B; ++b) {
    Fwd s;
    forward(P, x + kIn * b, round_bf16 != 0, s);
    y[b] = s.y;
  }
  return 0;
}

// Mean pinball loss at quantile tau of targets t and its gradient
// (5057) by back-propagation.  The GPU's BF16 rounding points are mirrored:
// the products of the backward pass use the rounded weights and
// activations, and the activation gradients dh2, dh1 are rounded to BF16
// before the weight-gradient sums (bias gradients use them unrounded).
int orc_mlp_loss_grad(const double* P, const float* x, const double* tgt, int64_t B, double tau,
                      int round_bf16, double* loss, double* grad) {
  const bool rnd = round_bf16 != 0;
  auto R = [&](double v) { return rnd ? bf16(v) : v; };
  std::vector<double> g(kParams, 0.0);
  double L = 0;
  std::vector<Fwd> S(B);
  for (int64_t b = 0; b < B; ++b) forward(P, x + kIn * b, rnd, S[b]);
  for (int64_t b = 0; b < B; ++b) {
    const Fwd& s = S[b];
    const double r = tgt[b] - s.y;
    L += r > 0 ? tau * r : (tau - 1.0) * r;
    const double dy = (r > 0 ? -tau : 1.0 - tau) / (double)B;
    g[oB3] += dy;
    double dh2[kH], dh1[kH];
    for (int k = 0; k < kH; ++k) {
      g[oW3 + k] += dy * s.h2[k];
      dh2[k] = s.a2[k] > 0 ? dy * R(P[oW3 + k]) : 0.0;
    }
    for (int k = 0; k < kH; ++k) {
      double a = 0;
      for (int j = 0; j < kH; ++j) a += R(P[oW2 + j * kH + k]) * R(dh2[j]);
      dh1[k] = s.a1[k] > 0 ? a : 0.0;
    }
    for (int j = 0; j < kH; ++j) {
      g[oB2 + j] += dh2[j];
      for (int k = 0; k < kH; ++k) g[oW2 + j * kH + k] += R(dh2[j]) * s.h1[k];
      g[oB1 + j] += dh1[j];
      for (int k = 0; k < kIn; ++k) g[oW1 + j * kIn + k] += R(dh1[j]) * s.x[k];
    }
  }
  *loss = L / (double)B;
  std::copy(g.begin(), g.end(), grad);
  return 0;
}

// One Adam step (Kingma & Ba, bias-corrected), step counted from 1.
int orc_adam(double* P, double* m, double* v, const double* g, int64_t n, double lr, double b1,
             double b2, double eps, int step) {
  const double c1 = 1.0 - std::pow(b1, step), c2 = 1.0 - std::pow(b2, step);
  for (int64_t i = 0; i < n; ++i) {
    m[i] = b1 * m[i] + (1.0 - b1) * g[i];
    v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
    P[i] -= lr * (m[i] / c1) / (std::sqrt(v[i] / c2) + eps);
  }
  return 0;
}

// Lists under the learned criterion of the selected groups (sel: group
// indices, NULL = every group in order), CSR in the order given.  Scores
// come from the network P (BF16 mirror) or, when P == NULL, from a replay
// table of (group index, cell id, score) triples sorted by (group, cell).
// fell_back (one per selected group, may be NULL) receives 1 for groups that
// fell back to theta.
static int learned_impl(const Tree& t, float theta, float th_lo, float th_hi, float log10_tau,
                        float budget, const double* P, const int32_t* rg, const int32_t* rc,
                        const float* rs, int64_t nr, int64_t* c_off, int32_t* c_ids,
                        int64_t* l_off, int32_t* l_ids, int64_t* n_c, int64_t* n_l,
                        int32_t* fell_back, const int32_t* sel, int64_t n_sel) {
  const int64_t ngt = (int64_t)t.groups.size();
  if (sel)
    for (int64_t u = 0; u < n_sel; ++u)
      if (sel[u] < 0 || sel[u] >= ngt) return -1;
  for (int64_t k = 0; k < nr; ++k)
    if (rg[k] < 0 || rg[k] >= ngt) return -1;
  const int64_t ng = sel ? n_sel : ngt;
  std::vector<std::vector<int32_t>> C(ng), Lv(ng);
  std::vector<int64_t> rbeg(ngt + 1, nr);
  if (!P) {  // index the replay table by group
    for (int64_t k = nr - 1; k >= 0; --k) rbeg[rg[k]] = k;
    for (int64_t u = ngt - 1; u >= 0; --u) rbeg[u] = std::min(rbeg[u], rbeg[u + 1]);
  }
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 8) reduction(| : bad)
  for (int64_t v = 0; v < ng; ++v) {
    const int64_t u = sel ? sel[v] : v;
    const int32_t gc = t.groups[u];
    auto score = [&](int32_t c) -> float {
      if (P) {
        float f[kIn];
        mac_features(t, gc, c, f);
        Fwd s;
        forward(P, f, true, s);
        return (float)s.y;
      }
      const int32_t* b = rc + rbeg[u];
      const int32_t* e = rc + rbeg[u + 1];
      const int32_t* it = std::lower_bound(b, e, c);
      if (it == e || *it != c) {
        bad = 1;
        return 0.0f;
      }
      return rs[it - rc];
    };
    const bool fb = walk_learned(t, gc, theta, th_lo, th_hi, log10_tau, budget, score, C[v], Lv[v]);
    if (fell_back) fell_back[v] = fb ? 1 : 0;
  }
  if (bad) return -2;  // a band candidate without a replayed score
  int64_t sc = 0, sl = 0;
  for (int64_t u = 0; u < ng; ++u) {
    if (c_off) c_off[u] = sc;
    if (l_off) l_off[u] = sl;
    if (c_ids) std::copy(C[u].begin(), C[u].end(), c_ids + sc);
    if (l_ids) std::copy(Lv[u].begin(), Lv[u].end(), l_ids + sl);
    sc += (int64_t)C[u].size();
    sl += (int64_t)Lv[u].size();
  }
  if (c_off) c_off[ng] = sc;
  if (l_off) l_off[ng] = sl;
  if (n_c) *n_c = sc;
  if (n_l) *n_l = sl;
  return 0;
}

// Lists of every group under the learned criterion (see learned_impl).
int orc_lists_learned(const void* h, float theta, float th_lo, float th_hi, float log10_tau,
                      float budget, const double* P, const int32_t* rg, const int32_t* rc,
                      const float* rs, int64_t nr, int64_t* c_off, int32_t* c_ids,
                      int64_t* l_off, int32_t* l_ids, int64_t* n_c, int64_t* n_l,
                      int32_t* fell_back) {
  return learned_impl(*(const Tree*)h, theta, th_lo, th_hi, log10_tau, budget, P, rg, rc, rs, nr,
                      c_off, c_ids, l_off, l_ids, n_c, n_l, fell_back, nullptr, -1);
}

// The same for the n_sel groups sel (group indices; the replay table's
// group column holds group indices too).
int orc_lists_learned_groups(const void* h, float theta, float th_lo, float th_hi,
                             float log10_tau, float budget, const double* P, const int32_t* rg,
                             const int32_t* rc, const float* rs, int64_t nr, const int32_t* sel,
                             int64_t n_sel, int64_t* c_off, int32_t* c_ids, int64_t* l_off,
                             int32_t* l_ids, int64_t* n_c, int64_t* n_l, int32_t* fell_back) {
  if (!sel || n_sel < 0) return -1;
  return learned_impl(*(const Tree*)h, theta, th_lo, th_hi, log10_tau, budget, P, rg, rc, rs, nr,
                      c_off, c_ids, l_off, l_ids, n_c, n_l, fell_back, sel, n_sel);
}

}  // extern "C"
