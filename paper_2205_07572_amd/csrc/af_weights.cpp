// af_weights.cpp -- host-side derivation of the fixed linear stencils of the
// AF point-value evolution.
//
// With constant coefficients and a fixed ratio dt/dx, the value of a node at
// t+tau is the same linear combination of the raw DOFs of the cells around
// it for every node of a kind (Sec. 2.1, Sec. 2.3).  Under 2:1 subcycling
// dt_l/dx_l is the same on every level, so one table serves all levels.
// This file computes those combinations once, in FP64, from:
//   * the biquadratic reconstruction (Sec. 2, eq. poly) in tensor Lagrange
//     form, whose centre value follows from "cell average = tensor Simpson
//     sum of the nodal values";
//   * advection (eq. advection-update): evaluation at the upwind foot;
//   * acoustics (eq. ERFormula, eq. sphe-mean): the spherical mean of each
//     cell polynomial over the disc sectors lying in that cell, integrated
//     in closed form monomial by monomial.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "af_internal.h"
#include "af_weights.h"

namespace af {
namespace {

constexpr double kPi = 3.141592653589793238462643383279502884;

// A biquadratic in reference coordinates: c[m][n] multiplies xi^m eta^n.
struct Poly2 {
  double c[3][3];
};

// 1D Lagrange basis on nodes -1, 0, 1 as monomial coefficients (power 0,1,2).
void lagrange_coeffs(int node, double out[3]) {
  if (node == -1) { out[0] = 0.0; out[1] = -0.5; out[2] = 0.5; }
  else if (node == 0) { out[0] = 1.0; out[1] = 0.0; out[2] = -1.0; }
  else { out[0] = 0.0; out[1] = 0.5; out[2] = 0.5; }
}

// Basis polynomial of raw DOF d (af_internal.h order) of one cell: the
// reconstruction equals sum_d dof_d * basis_d.  Nodal functions phi_ab =
// L_a(xi) L_b(eta); the centre value q00 = (36 avg - sum corners - 4 sum
// edges)/16 distributes phi_00 onto the raw DOFs.
Poly2 dof_basis(int d) {
  static const int node_of[9][2] = {{0, 0},  {-1, -1}, {1, -1}, {-1, 1}, {1, 1},
                                    {-1, 0}, {1, 0},   {0, -1}, {0, 1}};
  double lx[3], ly[3], cx[3], cy[3];
  lagrange_coeffs(0, cx);
  lagrange_coeffs(0, cy);
  Poly2 p;
  double centre_w;
  if (d == 0) {
    std::memset(p.c, 0, sizeof p.c);
    centre_w = 36.0 / 16.0;
  } else {
    lagrange_coeffs(node_of[d][0], lx);
    lagrange_coeffs(node_of[d][1], ly);
    for (int m = 0; m < 3; ++m)
      for (int n = 0; n < 3; ++n) p.c[m][n] = lx[m] * ly[n];
    centre_w = (d <= 4) ? -1.0 / 16.0 : -4.0 / 16.0;
  }
  for (int m = 0; m < 3; ++m)
    for (int n = 0; n < 3; ++n) p.c[m][n] += centre_w * cx[m] * cy[n];
  return p;
}

double poly_eval(const Poly2& p, double x, double y) {
  double s = 0.0, xm = 1.0;
  for (int m = 0; m < 3; ++m) {
    double yn = 1.0;
    for (int n = 0; n < 3; ++n) {
      s += p.c[m][n] * xm * yn;
      yn *= y;
    }
    xm *= x;
  }
  return s;
}

// Coefficients of p(x0 + s, y0 + t) in powers of (s, t).
Poly2 poly_shift(const Poly2& p, double x0, double y0) {
  static const double binom[3][3] = {{1, 0, 0}, {1, 1, 0}, {1, 2, 1}};
  Poly2 r;
  std::memset(r.c, 0, sizeof r.c);
  for (int m = 0; m < 3; ++m)
    for (int n = 0; n < 3; ++n)
      for (int a = m; a < 3; ++a)
        for (int b = n; b < 3; ++b)
          r.c[m][n] += p.c[a][b] * binom[a][m] * binom[b][n] * std::pow(x0, a - m) * std::pow(y0, b - n);
  return r;
}

// I(m,n) = int_0^{pi/2} cos^m(phi) sin^n(phi) dphi by the reduction
// I(m,n) = (m-1)/(m+n) I(m-2,n), I(m,n) = (n-1)/(m+n) I(m,n-2).
double trig_moment(int m, int n) {
  if (m >= 2) return double(m - 1) / double(m + n) * trig_moment(m - 2, n);
  if (n >= 2) return double(n - 1) / double(m + n) * trig_moment(m, n - 2);
  if (m == 0 && n == 0) return kPi / 2.0;
  if (m + n == 1) return 1.0;
  return 0.5;  // m = n = 1
}

// Angular moment over quadrant q (phi in [q pi/2, (q+1) pi/2]).
double quadrant_moment(int q, int m, int n) {
  double s = trig_moment(m, n);
  if ((q == 1 || q == 2) && (m & 1)) s = -s;  // cos < 0
  if ((q == 2 || q == 3) && (n & 1)) s = -s;  // sin < 0
  return s;
}

// Spherical mean, restricted to the quadrants in qmask, of a polynomial
// given in powers of the scaled displacement (zx/hx, zy/hy) about the disc
// centre: monomial (zx/hx)^m (zy/hy)^n contributes
//   (R/hx)^m (R/hy)^n I_{0,m+n+1} A_mn / (2 pi)
// (radial integral with s = R sin(theta)).  Returns M and R dM/dR.
void sector_mean(const double c[4][4], int qmask, double rx, double ry, double* M, double* RdM) {
  double sm = 0.0, sd = 0.0;
  for (int m = 0; m < 4; ++m)
    for (int n = 0; m + n < 6 && n < 4; ++n) {
      if (c[m][n] == 0.0) continue;
      double ang = 0.0;
      for (int q = 0; q < 4; ++q)
        if (qmask & (1 << q)) ang += quadrant_moment(q, m, n);
      const double rad = trig_moment(0, m + n + 1);
      const double mono = std::pow(rx, m) * std::pow(ry, n) * rad * ang / (2.0 * kPi);
      sm += c[m][n] * mono;
      sd += double(m + n) * c[m][n] * mono;
    }
  *M = sm;
  *RdM = sd;
}

// Advection: foot of the node in cell units relative to the owner cell's
// centre, then cell offset and reference coordinates.  A foot exactly on a
// face is put in the cell between it and the node.
void adv_locate(double node, double disp, int* off, double* ref) {
  const double s = node + disp;
  double k = std::floor(s + 0.5);
  if (disp > 0.0 && s + 0.5 == k) k -= 1.0;
  *off = int(k);
  *ref = 2.0 * (s - k);
}

// Rounds the FP64 weights w[0..n) of a stencil whose weights sum to
// `target` (1 for a value, 0 for a derivative: what a constant state
// requires) to T, keeping the rounded sum as close to the target as T
// allows.  Plain rounding leaves the FP32 sum off by up to a few 1e-8, and
// that error is systematic: every step scales a constant state by the same
// factor, so the mean drifts linearly with the step count (about 5e-5 after
// 1280 steps).  The residual is folded into the smallest weights, whose
// finer spacing then bounds it (an absolute change of the size of the
// rounding of the larger weights).  For T = double the weights are rounded
// plainly.
template <typename T>
void round_sum(const double* w, T* out, int n, double target) {
  for (int e = 0; e < n; ++e) out[e] = T(w[e]);
  if (sizeof(T) == sizeof(double)) return;
  for (int pass = 0; pass < 3; ++pass) {
    double sum = 0.0;  // exact: FP32 values spanning far fewer than 53 bits
    for (int e = 0; e < n; ++e) sum += double(out[e]);
    const double r = target - sum;
    if (r == 0.0) return;
    // smallest weight that the change leaves well away from zero
    int best = -1;
    for (int e = 0; e < n; ++e)
      if (std::fabs(w[e]) > 1e4 * std::fabs(r) && (best < 0 || std::fabs(w[e]) < std::fabs(w[best]))) best = e;
    if (best < 0) return;
    out[best] = T(double(out[best]) + r);
  }
}

}  // namespace

template <typename T>
void make_adv_weights(double a_dtdx, double b_dtdy, AdvWeights<T>* W) {
  static const double node_pos[3][2] = {{-0.5, -0.5}, {-0.5, 0.0}, {0.0, -0.5}};
  double wd[3][2][kCellDofs];
  bool up = true;
  for (int kind = 0; kind < 3; ++kind)
    for (int t = 0; t < 2; ++t) {
      const double frac = t == 0 ? 0.5 : 1.0;
      int ox, oy;
      double xi, eta;
      adv_locate(node_pos[kind][0], -a_dtdx * frac, &ox, &xi);
      adv_locate(node_pos[kind][1], -b_dtdy * frac, &oy, &eta);
      W->off[kind][t][0] = ox;
      W->off[kind][t][1] = oy;
      up = up && ox == (kind == 2 ? 0 : -1) && oy == (kind == 1 ? 0 : -1);
      for (int d = 0; d < kCellDofs; ++d) wd[kind][t][d] = poly_eval(dof_basis(d), xi, eta);
      round_sum(wd[kind][t], W->w[kind][t], kCellDofs, 1.0);
    }
  // Upwind pattern: compose the update of eq. 2dfv with the Simpson sums
  // (eq. Simpson-2d) of the eight face nodes of cell (0,0), each node's
  // half- and full-time values being its source cell's weights.
  double acc[25] = {};
  auto idx = [](int kind, int di, int dj) {
    switch (kind) {
      case 0: return kUpA + (dj + 1) * 2 + (di + 1);
      case 1: return kUpC + (dj + 1) * 3 + (di + 1);
      case 2: return kUpX + (dj + 1) * 3 + (di + 1);
      default: return kUpY + (dj + 1) * 2 + (di + 1);
    }
  };
  // raw DOF d of a cell: state kind and offset from the cell
  static const int dof_kind[9] = {0, 1, 1, 1, 1, 2, 2, 3, 3};
  static const int dof_off[9][2] = {{0, 0}, {0, 0}, {1, 0}, {0, 1}, {1, 1}, {0, 0}, {1, 0}, {0, 0}, {0, 1}};
  // adds c * (time sum of node kind nk owned by cell (oi, oj)) to acc
  auto add_tsum = [&](int nk, int oi, int oj, double c) {
    acc[idx(nk + 1, oi, oj)] += c;  // the node at time n
    const int si = oi + (nk == 2 ? 0 : -1), sj = oj + (nk == 1 ? 0 : -1);
    for (int d = 0; d < kCellDofs; ++d)
      acc[idx(dof_kind[d], si + dof_off[d][0], sj + dof_off[d][1])] += c * (4.0 * wd[nk][0][d] + wd[nk][1][d]);
  };
  const double cx = a_dtdx / 36.0, cy = b_dtdy / 36.0;
  acc[idx(0, 0, 0)] += 1.0;
  // -cx (FR - FL): FR over corner (1,0), x-edge (1,0), corner (1,1); FL over
  // corner (0,0), x-edge (0,0), corner (0,1); weights 1, 4, 1
  add_tsum(0, 1, 0, -cx); add_tsum(1, 1, 0, -4.0 * cx); add_tsum(0, 1, 1, -cx);
  add_tsum(0, 0, 0, cx); add_tsum(1, 0, 0, 4.0 * cx); add_tsum(0, 0, 1, cx);
  // -cy (GT - GB): GT over corner (0,1), y-edge (0,1), corner (1,1); GB over
  // corner (0,0), y-edge (0,0), corner (1,0)
  add_tsum(0, 0, 1, -cy); add_tsum(2, 0, 1, -4.0 * cy); add_tsum(0, 1, 1, -cy);
  add_tsum(0, 0, 0, cy); add_tsum(2, 0, 0, 4.0 * cy); add_tsum(0, 1, 0, cy);
  if (up)
    round_sum(acc, W->up_avg, 25, 1.0);
  else
    for (int e = 0; e < 25; ++e) W->up_avg[e] = T(0);
}

namespace {

// FP64 acoustic stencils D[tau][node kind][K, Dx, Dy][entry] (entries of the
// node kind's neighbourhood table), tau 0 = dt/2, 1 = dt.
void ac_dense(double c_dtdx, double c_dtdy, double D[2][3][3][kNbCorner]) {
  // node kind -> sectors: (quadrant mask, cell offset, node position in the
  // cell's reference coordinates)
  struct Sector { int qmask, di, dj; double xi, eta; };
  static const Sector corner_s[4] = {{1, 0, 0, -1, -1}, {2, -1, 0, 1, -1}, {4, -1, -1, 1, 1}, {8, 0, -1, -1, 1}};
  static const Sector xedge_s[2] = {{1 | 8, 0, 0, -1, 0}, {2 | 4, -1, 0, 1, 0}};
  static const Sector yedge_s[2] = {{1 | 2, 0, 0, 0, -1}, {4 | 8, 0, -1, 0, 1}};
  // raw DOF d of cell (di,dj) as (state kind, offset) relative to the owner
  static const int dof_kind[9] = {0, 1, 1, 1, 1, 2, 2, 3, 3};
  static const int dof_off[9][2] = {{0, 0}, {0, 0}, {1, 0}, {0, 1}, {1, 1}, {0, 0}, {1, 0}, {0, 0}, {0, 1}};

  for (int t = 0; t < 2; ++t) {
    const double frac = t == 0 ? 0.5 : 1.0;
    // scaled radii: R / (dx/2), R / (dy/2)
    const double rx = 2.0 * c_dtdx * frac, ry = 2.0 * c_dtdy * frac;
    for (int nk = 0; nk < 3; ++nk) {
      const Sector* secs = nk == 0 ? corner_s : (nk == 1 ? xedge_s : yedge_s);
      const int nsec = nk == 0 ? 4 : 2;
      const NbEntry* tab = nk == 0 ? kNbCornerTab : (nk == 1 ? kNbXedgeTab : kNbYedgeTab);
      const int nb = nk == 0 ? kNbCorner : kNbEdge;
      double (*acc)[kNbCorner] = D[t][nk];
      for (int w = 0; w < 3; ++w)
        for (int e = 0; e < kNbCorner; ++e) acc[w][e] = 0.0;
      for (int s = 0; s < nsec; ++s) {
        const Sector& S = secs[s];
        for (int d = 0; d < kCellDofs; ++d) {
          const Poly2 sh = poly_shift(dof_basis(d), S.xi, S.eta);
          // value, x-derivative and y-derivative (reference units, powers of
          // the scaled displacement) embedded in 4x4 coefficient grids
          double cv[4][4] = {}, cdx[4][4] = {}, cdy[4][4] = {};
          for (int m = 0; m < 3; ++m)
            for (int n = 0; n < 3; ++n) {
              cv[m][n] = sh.c[m][n];
              if (m > 0) cdx[m - 1][n] += double(m) * sh.c[m][n];
              if (n > 0) cdy[m][n - 1] += double(n) * sh.c[m][n];
            }
          double M, RdM, Mx, Rx, My, Ry;
          sector_mean(cv, S.qmask, rx, ry, &M, &RdM);
          sector_mean(cdx, S.qmask, rx, ry, &Mx, &Rx);
          sector_mean(cdy, S.qmask, rx, ry, &My, &Ry);
          // R d/dx = (R / (dx/2)) d/dxi = rx d/dxi
          const double K = M + RdM, Dx = rx * Mx, Dy = ry * My;
          const int kind = dof_kind[d];
          const int di = S.di + dof_off[d][0], dj = S.dj + dof_off[d][1];
          int e = 0;
          while (e < nb && !(tab[e].kind == kind && tab[e].di == di && tab[e].dj == dj)) ++e;
          acc[0][e] += K;
          acc[1][e] += Dx;
          acc[2][e] += Dy;
        }
      }
    }
  }
}

// round_sum for weights that enter a sum with multiplicities mult (the
// orbit sizes 1, 2, 4: exact scalings): the rounded sum of mult * w is kept
// as close to `target` as T allows.
// Each pass moves the one weight (of those well above the residual, so that
// the change is relatively tiny) whose rounded move leaves the smallest
// residual.
template <typename T>
void round_sum_mult(const double* w, const int* mult, T* out, int n, double target) {
  for (int e = 0; e < n; ++e) out[e] = T(w[e]);
  if (sizeof(T) == sizeof(double)) return;
  auto residual = [&]() {
    double sum = 0.0;  // exact: FP32 values times 1, 2 or 4
    for (int e = 0; e < n; ++e) sum += double(mult[e]) * double(out[e]);
    return target - sum;
  };
  for (int pass = 0; pass < 8; ++pass) {
    const double r = residual();
    if (r == 0.0) return;
    int best = -1;
    T best_val = T(0);
    double best_r = std::fabs(r);
    for (int e = 0; e < n; ++e) {
      if (!(std::fabs(w[e]) > 1e4 * std::fabs(r))) continue;
      const T keep = out[e];
      const T cand = T(double(keep) + r / double(mult[e]));
      out[e] = cand;
      const double nr = std::fabs(residual());
      out[e] = keep;
      if (nr < best_r) {
        best_r = nr;
        best = e;
        best_val = cand;
      }
    }
    if (best < 0) return;
    out[best] = best_val;
  }
}

int entry_index(int nk, const OrbitMember& mb) {
  for (int e = 0; e < nb_size(nk); ++e) {
    const NbEntry E = nb_entry(nk, e);
    if (E.kind == mb.kind && E.di == mb.di && E.dj == mb.dj) return e;
  }
  return -1;
}

}  // namespace

template <typename T>
void make_ac_weights(double c_dtdx, double c_dtdy, AcWeights<T>* W) {
  double D[2][3][3][kNbCorner];
  ac_dense(c_dtdx, c_dtdy, D);
  for (int t = 0; t < 2; ++t)
    for (int nk = 0; nk < 3; ++nk) {
      const int nb = nk == 0 ? kNbCorner : kNbEdge;
      // the spherical mean part sums to 1, the two gradient parts to 0
      for (int w = 0; w < 3; ++w) {
        T* dst = nk == 0 ? W->corner[t][w] : (nk == 1 ? W->xedge[t][w] : W->yedge[t][w]);
        round_sum(D[t][nk][w], dst, nb, w == 0 ? 1.0 : 0.0);
      }
    }
}

template <typename T>
bool make_ac_orbit_weights(double c_dtdx, double c_dtdy, AcOrbitWeights<T>* W) {
  double D[2][3][3][kNbCorner];
  ac_dense(c_dtdx, c_dtdy, D);
  double scale = 0.0;
  for (int t = 0; t < 2; ++t)
    for (int nk = 0; nk < 3; ++nk)
      for (int w = 0; w < 3; ++w)
        for (int e = 0; e < nb_size(nk); ++e) scale = std::max(scale, std::fabs(D[t][nk][w][e]));
  const double tol = 1e-12 * scale;
  bool ok = true;
  std::memset(W, 0, sizeof(*W));
  for (int nk = 0; nk < 3; ++nk) {
    const OrbitTable& OT = kOrbitTab[nk];
    // orbit weights per tau, then the two combinations
    double ow[2][kMaxOrbits][3] = {};
    for (int t = 0; t < 2; ++t)
      for (int o = 0; o < OT.n; ++o) {
        const NbOrbit& O = OT.o[o];
        for (int w = 0; w < 3; ++w) {
          double sum = 0.0;
          double val[4];
          for (int mb = 0; mb < O.n; ++mb) {
            int X = 0, Y = 0;
            nb_offset(nk, O.m[mb].kind, O.m[mb].di, O.m[mb].dj, &X, &Y);
            const double sg = w == 0 ? 1.0 : (w == 1 ? (X > 0 ? 1.0 : (X < 0 ? -1.0 : 0.0))
                                                     : (Y > 0 ? 1.0 : (Y < 0 ? -1.0 : 0.0)));
            const double d = D[t][nk][w][entry_index(nk, O.m[mb])];
            // a part odd in a direction with zero offset vanishes
            if (sg == 0.0 && std::fabs(d) > tol) ok = false;
            val[mb] = sg * d;
            sum += val[mb];
          }
          const bool present = w == 0 || (w == 1 && O.hasx) || (w == 2 && O.hasy);
          const double v = present ? sum / O.n : 0.0;
          for (int mb = 0; mb < O.n; ++mb)
            if (present && std::fabs(val[mb] - v) > tol) ok = false;
          ow[t][o][w] = v;
        }
      }
    // c = 0: value at t + dt; c = 1: 4 q(t + dt/2) + q(t + dt)
    for (int w = 0; w < 3; ++w)
      for (int c = 0; c < 2; ++c) {
        double src[kMaxOrbits];
        int mult[kMaxOrbits];
        for (int o = 0; o < OT.n; ++o) {
          src[o] = c == 0 ? ow[1][o][w] : 4.0 * ow[0][o][w] + ow[1][o][w];
          mult[o] = OT.o[o].n;
        }
        T out[kMaxOrbits];
        if (w == 0)
          round_sum_mult(src, mult, out, OT.n, c == 0 ? 1.0 : 5.0);
        else
          for (int o = 0; o < OT.n; ++o) out[o] = T(src[o]);
        for (int o = 0; o < OT.n; ++o) W->w[nk][o][c][w] = out[o];
      }
  }
  return ok;
}

void make_fill_weights(FillWeights* W) {
  // points: xi = cx/2 - 1, eta = cy/2 - 1
  for (int cy = 0; cy < 5; ++cy)
    for (int cx = 0; cx < 5; ++cx)
      for (int d = 0; d < kCellDofs; ++d) W->w[cx + 5 * cy][d] = poly_eval(dof_basis(d), 0.5 * cx - 1.0, 0.5 * cy - 1.0);
  // quarter [qx - 1, qx] x [qy - 1, qy]: tensor Simpson, exact for the biquadratic
  static const double sw[3] = {1.0, 4.0, 1.0};
  for (int qy = 0; qy < 2; ++qy)
    for (int qx = 0; qx < 2; ++qx)
      for (int d = 0; d < kCellDofs; ++d) {
        const Poly2 b = dof_basis(d);
        double s = 0.0;
        for (int p = 0; p < 3; ++p)
          for (int q = 0; q < 3; ++q) s += sw[p] * sw[q] * poly_eval(b, qx - 1.0 + 0.5 * p, qy - 1.0 + 0.5 * q);
        W->w[kFillPoints + qx + 2 * qy][d] = s / 36.0;
      }
}

template void make_adv_weights<float>(double, double, AdvWeights<float>*);
template void make_adv_weights<double>(double, double, AdvWeights<double>*);
template void make_ac_weights<float>(double, double, AcWeights<float>*);
template void make_ac_weights<double>(double, double, AcWeights<double>*);
template bool make_ac_orbit_weights<float>(double, double, AcOrbitWeights<float>*);
template bool make_ac_orbit_weights<double>(double, double, AcOrbitWeights<double>*);

}  // namespace af
