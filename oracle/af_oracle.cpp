// af_oracle.cpp -- reference (oracle) implementation of the Cartesian-grid
// Active Flux (AF) method with patch-based adaptive mesh refinement, after
// Calhoun, Chudzik & Helzel, "The Cartesian Grid Active Flux Method with
// Adaptive Mesh Refinement" (arXiv 2205.07572).
//
// TEST INFRASTRUCTURE ONLY.  This file is the slow, plain, FP64,
// single-threaded CPU oracle against which the GPU library is checked.  Only
// the test-suite, the smoke check and the CPU-baseline leg of the benchmark
// may load it.  It shares no code, header, table or constant generator with
// the GPU library, and the GPU library never calls it.
//
// Everything is written in the paper's notation and order:
//   * DOFs per cell (Sec. 2, last paragraph before Sec. 2.1): cell (i,j) owns
//     the average Q_ij, the left-edge midpoint Q_{i-1/2,j}, the bottom-left
//     corner Q_{i-1/2,j-1/2} and the bottom-edge midpoint Q_{i,j-1/2}.
//   * Reconstruction (Sec. 2, eq. poly): the biquadratic that interpolates the
//     eight boundary points and has the given average.  A biquadratic is
//     fixed by its 9 nodal values; the cell average of a biquadratic equals
//     the tensor Simpson sum of its nodal values, which fixes the centre
//     value.  We write it in tensor Lagrange form.
//   * Advection evolution (Sec. 2.1, eq. advection-update): evaluate q^n at
//     the upwind foot P - (a,b) tau.
//   * Acoustic evolution (Sec. 2.3, eq. ERFormula, eq. sphe-mean): the
//     Eymann-Roe formula evaluated exactly on the piecewise biquadratic q^n by
//     splitting the disc of radius R = c tau into the sectors that lie in the
//     adjacent cells (possible because of eq. cfl-acoustics) and integrating
//     the cell's Taylor polynomial about P over each sector in closed form.
//   * Variable-coefficient advection: solid-body rotation (Sec. 4.2, the node
//     turned back along its circle) and the swirl flow (Sec. 4.3, one RK4
//     step back in the field of the stream function).
//   * Burgers (Sec. 2.2, eq. burgers-sol, eq. Burgers-iterativ): two
//     fixed-point iterations from the mean of the neighbouring averages.
//   * Simpson space-time flux (Sec. 2, eq. Simpson-2d) and the finite-volume
//     update (eq. 2dfv).
//   * AMR (Sec. 3): quadtree of equal-size patches, 2:1 balance, two ghost
//     layers, fine->coarse and coarse->fine transfers (Sec. 3.1), subcycling
//     without time interpolation (Sec. 3.2) and the Berger-Colella
//     conservative fix (Sec. 3.2, "Global conservation property").
//
// Compile: g++ -O2 -ffp-contract=off -std=c++17 -shared -fPIC (no fast-math).

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

[[noreturn]] void die(const char* what) {
  std::fprintf(stderr, "af_oracle: %s\n", what);
  std::abort();
}

// ---------------------------------------------------------------------------
// Reconstruction (Sec. 2, eq. poly).
// ---------------------------------------------------------------------------

// 1D quadratic Lagrange basis on the reference interval [-1,1] with nodes
// -1, 0, 1, and its first and second derivatives.
double lag(int a, double s) {
  if (a == -1) return 0.5 * s * (s - 1.0);
  if (a == 0) return 1.0 - s * s;
  return 0.5 * s * (s + 1.0);
}
double lag_d1(int a, double s) {
  if (a == -1) return s - 0.5;
  if (a == 0) return -2.0 * s;
  return s + 0.5;
}
double lag_d2(int a) {
  if (a == 0) return -2.0;
  return 1.0;
}

// Nodal values of the reconstructed biquadratic of one cell: q[a+1][b+1] is
// the value at reference point (xi,eta) = (a,b), a,b in {-1,0,1}.
struct Cell {
  double q[3][3];
};

// Builds the cell polynomial from the average and the eight boundary points.
// The centre value follows from "average = Simpson sum of the nodal values":
//   Qbar = (sum corners + 4 sum edges + 16 q00) / 36.
Cell make_cell(double avg, double c_ll, double c_rl, double c_lu, double c_ru,
               double e_l, double e_r, double e_b, double e_t) {
  Cell c;
  c.q[0][0] = c_ll;
  c.q[2][0] = c_rl;
  c.q[0][2] = c_lu;
  c.q[2][2] = c_ru;
  c.q[0][1] = e_l;
  c.q[2][1] = e_r;
  c.q[1][0] = e_b;
  c.q[1][2] = e_t;
  c.q[1][1] = (36.0 * avg - (c_ll + c_rl + c_lu + c_ru) -
               4.0 * (e_l + e_r + e_b + e_t)) /
              16.0;
  return c;
}

double cell_eval(const Cell& c, double xi, double eta) {
  double s = 0.0;
  for (int a = -1; a <= 1; ++a)
    for (int b = -1; b <= 1; ++b) s += c.q[a + 1][b + 1] * lag(a, xi) * lag(b, eta);
  return s;
}

// Taylor coefficients of the cell polynomial about reference point
// (xi0,eta0), in PHYSICAL displacement units z = (zx,zy):
//   q(xi0 + 2 zx/dx, eta0 + 2 zy/dy) = sum_{m,n<=2} beta[m][n] zx^m zy^n.
void cell_taylor(const Cell& c, double xi0, double eta0, double dx, double dy,
                 double beta[3][3]) {
  for (int m = 0; m < 3; ++m)
    for (int n = 0; n < 3; ++n) beta[m][n] = 0.0;
  for (int a = -1; a <= 1; ++a) {
    const double tx[3] = {lag(a, xi0), lag_d1(a, xi0), 0.5 * lag_d2(a)};
    for (int b = -1; b <= 1; ++b) {
      const double ty[3] = {lag(b, eta0), lag_d1(b, eta0), 0.5 * lag_d2(b)};
      for (int m = 0; m < 3; ++m)
        for (int n = 0; n < 3; ++n) beta[m][n] += c.q[a + 1][b + 1] * tx[m] * ty[n];
    }
  }
  double sx = 1.0;
  for (int m = 0; m < 3; ++m) {
    double sy = 1.0;
    for (int n = 0; n < 3; ++n) {
      beta[m][n] *= sx * sy;
      sy *= 2.0 / dy;
    }
    sx *= 2.0 / dx;
  }
}

// ---------------------------------------------------------------------------
// Spherical mean over a quarter-disc sector (Sec. 2.3, eq. sphe-mean).
//
// For a monomial zx^m zy^n about the disc centre, with polar coordinates
// z = s (cos phi, sin phi) and the substitution s = R sin(theta):
//   (1/(2 pi R)) int_sector int_0^R s^{m+n} cos^m sin^n  s/sqrt(R^2-s^2) ds dphi
//     = R^{m+n} W_{m+n+1} A_mn(sector) / (2 pi),
//   W_k = int_0^{pi/2} sin^k(theta) dtheta,
//   A_mn(sector) = int_sector cos^m(phi) sin^n(phi) dphi.
// Quadrant q (0: phi in [0,pi/2], 1: [pi/2,pi], 2: [pi,3pi/2], 3: [3pi/2,2pi])
// relates to quadrant 0 by phi -> pi - phi, pi + phi, -phi.
// ---------------------------------------------------------------------------

double wallis(int k) {  // int_0^{pi/2} sin^k
  if (k == 0) return kPi / 2.0;
  if (k == 1) return 1.0;
  return wallis(k - 2) * double(k - 1) / double(k);
}

double a_q0(int m, int n) {  // int_0^{pi/2} cos^m sin^n, m,n <= 3
  // Beta-function closed form: 0.5 B((m+1)/2, (n+1)/2).
  return 0.5 * std::tgamma(0.5 * (m + 1)) * std::tgamma(0.5 * (n + 1)) /
         std::tgamma(0.5 * (m + n + 2));
}

// The constants W_k and A_mn(quadrant 0) are evaluated once from the closed
// forms above and kept in a table.
struct MeanTables {
  double w[6];
  double a[4][4];
  MeanTables() {
    for (int k = 0; k < 6; ++k) w[k] = wallis(k);
    for (int m = 0; m < 4; ++m)
      for (int n = 0; n < 4; ++n) a[m][n] = a_q0(m, n);
  }
};
const MeanTables& tables() {
  static const MeanTables t;
  return t;
}

double a_quad(int quad, int m, int n) {
  const double base = tables().a[m][n];
  const double sx = (m % 2) ? -1.0 : 1.0;
  const double sy = (n % 2) ? -1.0 : 1.0;
  switch (quad) {
    case 0: return base;
    case 1: return sx * base;
    case 2: return sx * sy * base;
    default: return sy * base;
  }
}

// Sector spherical mean of a polynomial given by its Taylor coefficients
// coef[m][n] (m,n < 4) about the disc centre, together with R d/dR of it.
void sector_mean(const double coef[4][4], int quad, double R, double* mean,
                 double* r_dmean) {
  double s = 0.0, sd = 0.0;
  double rp[7] = {1.0, 0, 0, 0, 0, 0, 0};
  for (int k = 1; k < 7; ++k) rp[k] = rp[k - 1] * R;
  for (int m = 0; m < 4; ++m)
    for (int n = 0; n < 4; ++n) {
      if (coef[m][n] == 0.0) continue;
      const double mono = rp[m + n] * tables().w[m + n + 1] * a_quad(quad, m, n) / (2.0 * kPi);
      s += coef[m][n] * mono;
      sd += coef[m][n] * double(m + n) * mono;
    }
  *mean = s;
  *r_dmean = sd;
}

// ---------------------------------------------------------------------------
// Access to DOF arrays.  A Grid maps cell/node indices of one Cartesian grid
// to storage.  Two implementations: a periodic single grid, and one patch
// block (interior m x m plus g ghost layers; indices outside the block abort).
// ---------------------------------------------------------------------------

enum Kind { K_AVG = 0, K_CORNER = 1, K_XEDGE = 2, K_YEDGE = 3 };

struct Grid {
  int ncomp = 1;
  double dx = 1.0, dy = 1.0;
  double ox = 0.0, oy = 0.0;  // physical position of the left / bottom face of cell 0
  virtual ~Grid() = default;
  virtual double get(int kind, int comp, int i, int j) const = 0;
  Cell cell(int comp, int i, int j) const {
    return make_cell(get(K_AVG, comp, i, j), get(K_CORNER, comp, i, j),
                     get(K_CORNER, comp, i + 1, j), get(K_CORNER, comp, i, j + 1),
                     get(K_CORNER, comp, i + 1, j + 1), get(K_XEDGE, comp, i, j),
                     get(K_XEDGE, comp, i + 1, j), get(K_YEDGE, comp, i, j),
                     get(K_YEDGE, comp, i, j + 1));
  }
};

// Periodic Nx x Ny grid; each array is [ncomp][Ny][Nx]; corner (i,j) is the
// node (x_{i-1/2}, y_{j-1/2}), xedge (i,j) is (x_{i-1/2}, y_j), yedge (i,j) is
// (x_i, y_{j-1/2}).
struct PeriodicGrid : Grid {
  int nx = 0, ny = 0;
  const double* arr[4] = {nullptr, nullptr, nullptr, nullptr};
  double get(int kind, int comp, int i, int j) const override {
    i = ((i % nx) + nx) % nx;
    j = ((j % ny) + ny) % ny;
    return arr[kind][(size_t(comp) * ny + j) * nx + i];
  }
};

// One patch block: every kind is stored in a (S+1) x (S+1) plane per
// component, S = m + 2g, row index j+g, column index i+g.  Valid index ranges
// (local, interior cells are [0,m)):  avg i,j in [-g, m+g);  corner
// i,j in [-g, m+g];  xedge i in [-g, m+g], j in [-g, m+g);  yedge i in
// [-g, m+g), j in [-g, m+g].
struct BlockGrid : Grid {
  int m = 0, g = 2;
  const double* arr[4] = {nullptr, nullptr, nullptr, nullptr};
  int plane() const { return (m + 2 * g + 1) * (m + 2 * g + 1); }
  bool valid(int kind, int i, int j) const {
    const int lo = -g, hc = m + g, hn = m + g + 1;
    const int ix_hi = (kind == K_AVG || kind == K_YEDGE) ? hc : hn;
    const int jy_hi = (kind == K_AVG || kind == K_XEDGE) ? hc : hn;
    return i >= lo && i < ix_hi && j >= lo && j < jy_hi;
  }
  size_t idx(int comp, int i, int j) const {
    const int P = m + 2 * g + 1;
    return size_t(comp) * plane() + size_t(j + g) * P + size_t(i + g);
  }
  double get(int kind, int comp, int i, int j) const override {
    if (!valid(kind, i, j)) die("block read outside the patch block");
    return arr[kind][idx(comp, i, j)];
  }
};

// ---------------------------------------------------------------------------
// Point-value evolution (Sec. 2.1 and Sec. 2.3).
// A node is identified by its kind and owning cell (i,j) (Sec. 2 ownership).
// Its position in "cell units" (cell k spans [k-1/2, k+1/2]) is
//   corner (i-1/2, j-1/2), xedge (i-1/2, j), yedge (i, j-1/2).
// ---------------------------------------------------------------------------

struct Physics {
  int eq = 0;            // 0 advection, 1 acoustics, 2 solid-body rotation, 3 swirl, 4 Burgers
  double a = 0, b = 0;   // advection velocity
  double c = 1;          // speed of sound
  double omega = 0, xc = 0, yc = 0;  // rotation: a = -omega (y - yc), b = omega (x - xc)
  double t = 0;          // time at the start of the step (swirl)
  int iters = 2;         // Burgers: fixed-point iterations per point value
};

void node_pos(int kind, int i, int j, double* X, double* Y) {
  *X = (kind == K_YEDGE) ? double(i) : double(i) - 0.5;
  *Y = (kind == K_XEDGE) ? double(j) : double(j) - 0.5;
}

// Cell containing coordinate s (cell units) of a foot traced back with
// velocity vel, and the reference coordinate in it.  A foot lying exactly on
// a cell face is assigned to the cell between the foot and the node it was
// traced from, which keeps it inside the one-cell stencil when CFL = 1; the
// reconstruction is continuous, so the choice does not change the value.
void locate(double s, double vel, int* k, double* ref) {
  double kk;
  if (vel < 0.0) {
    kk = std::ceil(s + 0.5) - 1.0;  // s in (k-1/2, k+1/2]
  } else {
    kk = std::floor(s + 0.5);  // s in [k-1/2, k+1/2)
  }
  *k = int(kk);
  *ref = 2.0 * (s - kk);
}

// Advection (eq. advection-update): q^n at the foot P - (a,b) tau.
double advect_point(const Grid& g, const Physics& ph, int kind, int i, int j, double tau) {
  double X, Y;
  node_pos(kind, i, j, &X, &Y);
  const double fx = X - ph.a * tau / g.dx;
  const double fy = Y - ph.b * tau / g.dy;
  int ci, cj;
  double xi, eta;
  locate(fx, ph.a, &ci, &xi);
  locate(fy, ph.b, &cj, &eta);
  return cell_eval(g.cell(0, ci, cj), xi, eta);
}

// Physical position of a node (cell units X, Y as in node_pos).
void node_xy(const Grid& g, int kind, int i, int j, double* x, double* y) {
  double X, Y;
  node_pos(kind, i, j, &X, &Y);
  *x = g.ox + (X + 0.5) * g.dx;
  *y = g.oy + (Y + 0.5) * g.dy;
}

// Velocity components of the advecting field at a physical point.
double vel_a(const Physics& ph, double x, double y) { (void)x; return ph.eq == 2 ? -ph.omega * (y - ph.yc) : ph.a; }
double vel_b(const Physics& ph, double x, double y) { (void)y; return ph.eq == 2 ? ph.omega * (x - ph.xc) : ph.b; }

// Solid-body rotation (Sec. 4.2): the characteristic through the node is a
// circle about (xc, yc); its position a time tau earlier is the node turned
// by -omega tau (eq. characteristics_advtwo with t = -tau), and q^n is
// evaluated there.  A foot on a face goes to the cell between foot and node,
// as for constant advection.
double rotate_point(const Grid& g, const Physics& ph, int kind, int i, int j, double tau) {
  double x, y;
  node_xy(g, kind, i, j, &x, &y);
  const double th = ph.omega * tau;
  const double rx = x - ph.xc, ry = y - ph.yc;
  const double fx = ph.xc + rx * std::cos(th) + ry * std::sin(th);
  const double fy = ph.yc - rx * std::sin(th) + ry * std::cos(th);
  const double sx = (fx - g.ox) / g.dx - 0.5, sy = (fy - g.oy) / g.dy - 0.5;  // cell units
  int ci, cj;
  double xi, eta;
  locate(sx, x - fx, &ci, &xi);
  locate(sy, y - fy, &cj, &eta);
  return cell_eval(g.cell(0, ci, cj), xi, eta);
}

// Swirl flow (Sec. 4.3): stream function
//   Psi(x, y, t) = sin^2(pi x) sin^2(pi y) cos(pi t) / pi
// and the velocity of eq. swirlODE, its centred differences over one cell of
// the grid the step runs on.
double swirl_psi(double x, double y, double t) {
  const double sx = std::sin(kPi * x), sy = std::sin(kPi * y);
  return sx * sx * sy * sy * std::cos(kPi * t) / kPi;
}
void swirl_vel(const Grid& g, double x, double y, double t, double* a, double* b) {
  *a = -(swirl_psi(x, y + 0.5 * g.dy, t) - swirl_psi(x, y - 0.5 * g.dy, t)) / g.dy;
  *b = (swirl_psi(x + 0.5 * g.dx, y, t) - swirl_psi(x - 0.5 * g.dx, y, t)) / g.dx;
}

// The characteristic through (x, y) at time t + tau traced back to t by one
// step of the classical fourth-order Runge-Kutta method (Sec. 4.3).
void swirl_trace(const Grid& g, double x, double y, double t, double tau, double* fx, double* fy) {
  const double t1 = t + tau, h = -tau;
  double a1, b1, a2, b2, a3, b3, a4, b4;
  swirl_vel(g, x, y, t1, &a1, &b1);
  swirl_vel(g, x + 0.5 * h * a1, y + 0.5 * h * b1, t1 + 0.5 * h, &a2, &b2);
  swirl_vel(g, x + 0.5 * h * a2, y + 0.5 * h * b2, t1 + 0.5 * h, &a3, &b3);
  swirl_vel(g, x + h * a3, y + h * b3, t1 + h, &a4, &b4);
  *fx = x + h / 6.0 * (a1 + 2.0 * a2 + 2.0 * a3 + a4);
  *fy = y + h / 6.0 * (b1 + 2.0 * b2 + 2.0 * b3 + b4);
}

// q^n at the foot of the node's characteristic (Sec. 4.3).
double swirl_point(const Grid& g, const Physics& ph, int kind, int i, int j, double tau) {
  double x, y, fx, fy;
  node_xy(g, kind, i, j, &x, &y);
  swirl_trace(g, x, y, ph.t, tau, &fx, &fy);
  const double sx = (fx - g.ox) / g.dx - 0.5, sy = (fy - g.oy) / g.dy - 0.5;
  int ci, cj;
  double xi, eta;
  locate(sx, x - fx, &ci, &xi);
  locate(sy, y - fy, &cj, &eta);
  return cell_eval(g.cell(0, ci, cj), xi, eta);
}

// Burgers (Sec. 2.2).  For smooth solutions the point value solves the
// implicit relation q(P, t + tau) = q^n(P - q(P, t + tau) tau (1, 1))
// (eq. burgers-sol).  It is found by fixed-point iteration (eq.
// Burgers-iterativ): the starting speed is the mean of the cell averages
// around the node (four for a corner, the two cells the edge separates for an
// edge midpoint), and each iteration evaluates q^n at the foot of the current
// speed.  `iters` iterations (two give third order).
double burgers_point(const Grid& g, const Physics& ph, int kind, int i, int j, double tau) {
  double Q;
  if (kind == K_CORNER) {
    Q = 0.25 * (g.get(K_AVG, 0, i - 1, j) + g.get(K_AVG, 0, i, j) + g.get(K_AVG, 0, i - 1, j - 1) +
                g.get(K_AVG, 0, i, j - 1));
  } else if (kind == K_XEDGE) {  // (x_{i-1/2}, y_j) between cells (i-1, j) and (i, j)
    Q = 0.5 * (g.get(K_AVG, 0, i - 1, j) + g.get(K_AVG, 0, i, j));
  } else {  // yedge (x_i, y_{j-1/2}) between cells (i, j) and (i, j-1)
    Q = 0.5 * (g.get(K_AVG, 0, i, j) + g.get(K_AVG, 0, i, j - 1));
  }
  double X, Y;
  node_pos(kind, i, j, &X, &Y);
  for (int it = 0; it < ph.iters; ++it) {
    const double fx = X - Q * tau / g.dx, fy = Y - Q * tau / g.dy;
    int ci, cj;
    double xi, eta;
    locate(fx, Q, &ci, &xi);
    locate(fy, Q, &cj, &eta);
    Q = cell_eval(g.cell(0, ci, cj), xi, eta);
  }
  return Q;
}

// Acoustics (eq. ERFormula with R = c tau):
//   p = M{p} + R dM{p}/dR - R M{div u},
//   u = M{u} + R dM{u}/dR - R M{p_x},  v = M{v} + R dM{v}/dR - R M{p_y}.
// The disc around a corner is split into the four quadrants lying in the four
// cells meeting there; around an edge midpoint into two half discs (each the
// union of two quadrants) lying in the two adjacent cells.  On each sector
// the integrand is that cell's polynomial, expanded about P.
void acoustic_point(const Grid& g, const Physics& ph, int kind, int i, int j, double tau,
                    double out[3]) {
  const double R = ph.c * tau;
  // (quadrant, cell offset di, dj, reference coords of P in that cell)
  struct Sec { int quad, ci, cj; double xi0, eta0; };
  Sec secs[4];
  if (kind == K_CORNER) {
    secs[0] = {0, i, j, -1.0, -1.0}; secs[1] = {1, i - 1, j, 1.0, -1.0};
    secs[2] = {2, i - 1, j - 1, 1.0, 1.0}; secs[3] = {3, i, j - 1, -1.0, 1.0};
  } else if (kind == K_XEDGE) {  // P = (x_{i-1/2}, y_j): right half in cell (i,j)
    secs[0] = {0, i, j, -1.0, 0.0}; secs[1] = {3, i, j, -1.0, 0.0};
    secs[2] = {1, i - 1, j, 1.0, 0.0}; secs[3] = {2, i - 1, j, 1.0, 0.0};
  } else {  // yedge, P = (x_i, y_{j-1/2}): top half in cell (i,j)
    secs[0] = {0, i, j, 0.0, -1.0}; secs[1] = {1, i, j, 0.0, -1.0};
    secs[2] = {2, i, j - 1, 0.0, 1.0}; secs[3] = {3, i, j - 1, 0.0, 1.0};
  }
  double p = 0.0, u = 0.0, v = 0.0;
  for (const Sec& s : secs) {
    double bp[3][3], bu[3][3], bv[3][3];
    cell_taylor(g.cell(0, s.ci, s.cj), s.xi0, s.eta0, g.dx, g.dy, bp);
    cell_taylor(g.cell(1, s.ci, s.cj), s.xi0, s.eta0, g.dx, g.dy, bu);
    cell_taylor(g.cell(2, s.ci, s.cj), s.xi0, s.eta0, g.dx, g.dy, bv);
    double cp[4][4] = {}, cu[4][4] = {}, cv[4][4] = {};
    double cdiv[4][4] = {}, cpx[4][4] = {}, cpy[4][4] = {};
    for (int m = 0; m < 3; ++m)
      for (int n = 0; n < 3; ++n) {
        cp[m][n] = bp[m][n];
        cu[m][n] = bu[m][n];
        cv[m][n] = bv[m][n];
        // derivative of zx^m zy^n
        if (m > 0) {
          cdiv[m - 1][n] += double(m) * bu[m][n];
          cpx[m - 1][n] += double(m) * bp[m][n];
        }
        if (n > 0) {
          cdiv[m][n - 1] += double(n) * bv[m][n];
          cpy[m][n - 1] += double(n) * bp[m][n];
        }
      }
    double M, RdM, Md, unused;
    sector_mean(cp, s.quad, R, &M, &RdM);
    sector_mean(cdiv, s.quad, R, &Md, &unused);
    p += M + RdM - R * Md;
    sector_mean(cu, s.quad, R, &M, &RdM);
    sector_mean(cpx, s.quad, R, &Md, &unused);
    u += M + RdM - R * Md;
    sector_mean(cv, s.quad, R, &M, &RdM);
    sector_mean(cpy, s.quad, R, &Md, &unused);
    v += M + RdM - R * Md;
  }
  out[0] = p;
  out[1] = u;
  out[2] = v;
}

void evolve_point(const Grid& g, const Physics& ph, int kind, int i, int j, double tau,
                  double out[3]) {
  if (ph.eq == 0) {
    out[0] = advect_point(g, ph, kind, i, j, tau);
  } else if (ph.eq == 2) {
    out[0] = rotate_point(g, ph, kind, i, j, tau);
  } else if (ph.eq == 3) {
    out[0] = swirl_point(g, ph, kind, i, j, tau);
  } else if (ph.eq == 4) {
    out[0] = burgers_point(g, ph, kind, i, j, tau);
  } else {
    acoustic_point(g, ph, kind, i, j, tau, out);
  }
}

// Physical flux functions: advection f = a q, g = b q with the velocity
// component at the node (constant, or that of the rotation field, Sec. 4.2);
// acoustics f = c (u, p, 0), g = c (v, 0, p) for q = (p, u, v) (Sec. 2.3);
// Burgers f = g = q^2 / 2 (eq. burgers2d).
void flux_x(const Physics& ph, double vel, const double* q, double* f) {
  if (ph.eq == 4) {
    f[0] = 0.5 * q[0] * q[0];
  } else if (ph.eq != 1) {
    f[0] = vel * q[0];
  } else {
    f[0] = ph.c * q[1];
    f[1] = ph.c * q[0];
    f[2] = 0.0;
  }
}
void flux_y(const Physics& ph, double vel, const double* q, double* f) {
  if (ph.eq == 4) {
    f[0] = 0.5 * q[0] * q[0];
  } else if (ph.eq != 1) {
    f[0] = vel * q[0];
  } else {
    f[0] = ph.c * q[2];
    f[1] = 0.0;
    f[2] = ph.c * q[0];
  }
}

// Simpson space-time flux (eq. Simpson-2d): nodes lo/mid/hi along the face at
// times n, n+1/2, n+1, weights (1,4,1) x (1,4,1) / 36.  vel: the normal
// velocity at the nine points in the same order (advection-type equations).
void simpson_flux(const Physics& ph, bool xface, const double vel[9], const double* n_lo,
                  const double* n_mid, const double* n_hi, const double* h_lo, const double* h_mid,
                  const double* h_hi, const double* f_lo, const double* f_mid,
                  const double* f_hi, int ncomp, double* F) {
  const double* pts[9] = {n_lo, n_mid, n_hi, h_lo, h_mid, h_hi, f_lo, f_mid, f_hi};
  const double w[9] = {1, 4, 1, 4, 16, 4, 1, 4, 1};
  for (int c = 0; c < ncomp; ++c) F[c] = 0.0;
  for (int k = 0; k < 9; ++k) {
    double f[3];
    if (xface) flux_x(ph, vel[k], pts[k], f); else flux_y(ph, vel[k], pts[k], f);
    for (int c = 0; c < ncomp; ++c) F[c] += w[k] * f[c];
  }
  for (int c = 0; c < ncomp; ++c) F[c] /= 36.0;
}

// Normal velocity at the nine Simpson points of the x-face at x_{i-1/2}, row
// j (xface) or of the y-face at y_{j-1/2}, column i, ordered (time n, n+1/2,
// n+1) x (lo, mid, hi node): constant; the rotation field at each node
// (Sec. 4.2); or, for the swirl (eq. flux_swirl, eq. swirlF/G), the field at
// the face midpoint at each of the three times.
void face_velocities(const Grid& g, const Physics& ph, bool xface, int i, int j, double dt, double vel[9]) {
  const int kind_lo = K_CORNER, kind_mid = xface ? K_XEDGE : K_YEDGE;
  const int il = i, jl = j, ih = xface ? i : i + 1, jh = xface ? j + 1 : j;
  double x[3], y[3];
  node_xy(g, kind_lo, il, jl, &x[0], &y[0]);
  node_xy(g, kind_mid, i, j, &x[1], &y[1]);
  node_xy(g, kind_lo, ih, jh, &x[2], &y[2]);
  for (int tl = 0; tl < 3; ++tl)
    for (int n = 0; n < 3; ++n) {
      double v;
      if (ph.eq == 3) {
        double a, b;
        swirl_vel(g, x[1], y[1], ph.t + 0.5 * tl * dt, &a, &b);
        v = xface ? a : b;
      } else {
        v = xface ? vel_a(ph, x[n], y[n]) : vel_b(ph, x[n], y[n]);
      }
      vel[3 * tl + n] = v;
    }
}

// ---------------------------------------------------------------------------
// One AF time step on a cell range [i0,i1) x [j0,j1) of a grid.
// Computes the new point values of every node on the boundary of the range
// (node index ranges [i0,i1] x [j0,j1]) at t+dt/2 and t+dt, the Simpson
// fluxes of every face of the range, and the updated averages (eq. 2dfv).
// Results are returned through callbacks-free plain vectors indexed relative
// to (i0, j0).
// ---------------------------------------------------------------------------

struct StepResult {
  int i0, j0, ni, nj, ncomp;
  // node values at t+dt for node (i,j), i in [i0,i0+ni], j in [j0,j0+nj]
  std::vector<double> corner, xedge, yedge;  // [(j-j0)*(ni+1)+(i-i0)][comp]
  std::vector<double> avg;                   // [(j-j0)*ni+(i-i0)][comp]
  std::vector<double> Fx;                    // x-face at x_{i-1/2}, row j: [(j-j0)*(ni+1)+(i-i0)][comp]
  std::vector<double> Gy;                    // y-face at y_{j-1/2}, col i: [(j-j0)*ni+(i-i0)][comp]
};

StepResult af_step_range(const Grid& g, const Physics& ph, double dt, int i0, int i1, int j0,
                         int j1) {
  const int nc = g.ncomp;
  const int ni = i1 - i0, nj = j1 - j0;
  const int NI = ni + 1, NJ = nj + 1;  // node lattice extents
  StepResult r;
  r.i0 = i0; r.j0 = j0; r.ni = ni; r.nj = nj; r.ncomp = nc;
  // point values at n (current), n+1/2, n+1 for each node kind on the lattice
  std::vector<double> cur[4], half[4], full[4];
  for (int k = 1; k < 4; ++k) {
    cur[k].assign(size_t(NI) * NJ * nc, 0.0);
    half[k].assign(size_t(NI) * NJ * nc, 0.0);
    full[k].assign(size_t(NI) * NJ * nc, 0.0);
  }
  auto nid = [&](int i, int j) { return (size_t(j - j0) * NI + size_t(i - i0)) * nc; };
  for (int j = j0; j <= j1; ++j)
    for (int i = i0; i <= i1; ++i)
      for (int kind = 1; kind < 4; ++kind) {
        // only nodes that lie on the boundary of some cell of the range
        if (kind == K_XEDGE && j == j1) continue;
        if (kind == K_YEDGE && i == i1) continue;
        double oh[3] = {0, 0, 0}, of[3] = {0, 0, 0};
        evolve_point(g, ph, kind, i, j, 0.5 * dt, oh);
        evolve_point(g, ph, kind, i, j, dt, of);
        for (int c = 0; c < nc; ++c) {
          cur[kind][nid(i, j) + c] = g.get(kind, c, i, j);
          half[kind][nid(i, j) + c] = oh[c];
          full[kind][nid(i, j) + c] = of[c];
        }
      }
  // fluxes
  r.Fx.assign(size_t(NI) * nj * nc, 0.0);
  r.Gy.assign(size_t(ni) * NJ * nc, 0.0);
  for (int j = j0; j < j1; ++j)
    for (int i = i0; i <= i1; ++i) {
      // x-face at x_{i-1/2}, y in [y_{j-1/2}, y_{j+1/2}]: corner (i,j), xedge (i,j), corner (i,j+1)
      double vel[9];
      face_velocities(g, ph, true, i, j, dt, vel);
      simpson_flux(ph, true, vel, &cur[K_CORNER][nid(i, j)], &cur[K_XEDGE][nid(i, j)],
                   &cur[K_CORNER][nid(i, j + 1)], &half[K_CORNER][nid(i, j)],
                   &half[K_XEDGE][nid(i, j)], &half[K_CORNER][nid(i, j + 1)],
                   &full[K_CORNER][nid(i, j)], &full[K_XEDGE][nid(i, j)],
                   &full[K_CORNER][nid(i, j + 1)], nc,
                   &r.Fx[(size_t(j - j0) * NI + size_t(i - i0)) * nc]);
    }
  for (int j = j0; j <= j1; ++j)
    for (int i = i0; i < i1; ++i) {
      // y-face at y_{j-1/2}: corner (i,j), yedge (i,j), corner (i+1,j)
      double vel[9];
      face_velocities(g, ph, false, i, j, dt, vel);
      simpson_flux(ph, false, vel, &cur[K_CORNER][nid(i, j)], &cur[K_YEDGE][nid(i, j)],
                   &cur[K_CORNER][nid(i + 1, j)], &half[K_CORNER][nid(i, j)],
                   &half[K_YEDGE][nid(i, j)], &half[K_CORNER][nid(i + 1, j)],
                   &full[K_CORNER][nid(i, j)], &full[K_YEDGE][nid(i, j)],
                   &full[K_CORNER][nid(i + 1, j)], nc,
                   &r.Gy[(size_t(j - j0) * ni + size_t(i - i0)) * nc]);
    }
  // conservative update (eq. 2dfv)
  r.avg.assign(size_t(ni) * nj * nc, 0.0);
  for (int j = j0; j < j1; ++j)
    for (int i = i0; i < i1; ++i)
      for (int c = 0; c < nc; ++c) {
        const double FL = r.Fx[(size_t(j - j0) * NI + size_t(i - i0)) * nc + c];
        const double FR = r.Fx[(size_t(j - j0) * NI + size_t(i + 1 - i0)) * nc + c];
        const double GB = r.Gy[(size_t(j - j0) * ni + size_t(i - i0)) * nc + c];
        const double GT = r.Gy[(size_t(j + 1 - j0) * ni + size_t(i - i0)) * nc + c];
        r.avg[(size_t(j - j0) * ni + size_t(i - i0)) * nc + c] =
            g.get(K_AVG, c, i, j) - dt / g.dx * (FR - FL) - dt / g.dy * (GT - GB);
      }
  r.corner = full[K_CORNER];
  r.xedge = full[K_XEDGE];
  r.yedge = full[K_YEDGE];
  return r;
}

// ---------------------------------------------------------------------------
// Patch-based AMR (Sec. 3).
// ---------------------------------------------------------------------------

struct Leaf {
  int level = 0, ix = 0, iy = 0;
  std::vector<double> blk[4];  // [ncomp][(S+1)^2] per kind
  std::vector<double> reg;     // flux register [4 sides][m][ncomp]: sum of F * face length * dt
};

enum Side { S_W = 0, S_E = 1, S_S = 2, S_N = 3 };

struct Hier {
  Physics ph;
  double time = 0.0;  // time of the synchronised state
  int m = 16, g = 2, ncomp = 1;
  int n0x = 1, n0y = 1, lmax = 0;
  double x0 = 0, y0 = 0, lx = 1, ly = 1;
  std::vector<Leaf> leaves;
  std::map<std::tuple<int, int, int>, int> index;

  int S1() const { return m + 2 * g + 1; }
  size_t plane() const { return size_t(S1()) * S1(); }
  int npx(int l) const { return n0x << l; }
  int npy(int l) const { return n0y << l; }
  double dx(int l) const { return lx / double(n0x * m) / double(1 << l); }
  double dy(int l) const { return ly / double(n0y * m) / double(1 << l); }

  void reindex() {
    index.clear();
    for (int k = 0; k < int(leaves.size()); ++k)
      index[{leaves[k].level, leaves[k].ix, leaves[k].iy}] = k;
  }
  int find(int l, int px, int py) const {
    if (l < 0 || l > 30) return -1;
    const int nx = npx(l), ny = npy(l);
    px = ((px % nx) + nx) % nx;
    py = ((py % ny) + ny) % ny;
    auto it = index.find({l, px, py});
    return it == index.end() ? -1 : it->second;
  }
  size_t bidx(int comp, int i, int j) const {
    return size_t(comp) * plane() + size_t(j + g) * S1() + size_t(i + g);
  }
  double& at(Leaf& L, int kind, int comp, int i, int j) { return L.blk[kind][bidx(comp, i, j)]; }
  double at(const Leaf& L, int kind, int comp, int i, int j) const {
    return L.blk[kind][bidx(comp, i, j)];
  }
  void alloc(Leaf& L) const {
    for (int k = 0; k < 4; ++k) L.blk[k].assign(plane() * ncomp, 0.0);
    L.reg.assign(size_t(4) * m * ncomp, 0.0);
  }
  BlockGrid view(const Leaf& L) const {
    BlockGrid bg;
    bg.m = m; bg.g = g; bg.ncomp = ncomp;
    bg.dx = dx(L.level); bg.dy = dy(L.level);
    bg.ox = x0 + L.ix * m * bg.dx;
    bg.oy = y0 + L.iy * m * bg.dy;
    for (int k = 0; k < 4; ++k) bg.arr[k] = L.blk[k].data();
    return bg;
  }
};

// Closed-square test of two leaves with periodic wrap (used for 2:1 balance
// with corner adjacency).  Coordinates in units of finest-level cells.
bool touches(const Hier& h, const Leaf& A, const Leaf& B, int lref) {
  const long long NX = (long long)h.n0x * h.m << lref, NY = (long long)h.n0y * h.m << lref;
  auto span = [&](const Leaf& L, long long* x0, long long* x1, long long* y0, long long* y1) {
    const long long w = (long long)h.m << (lref - L.level);
    *x0 = L.ix * w; *x1 = *x0 + w;
    *y0 = L.iy * w; *y1 = *y0 + w;
  };
  long long ax0, ax1, ay0, ay1, bx0, bx1, by0, by1;
  span(A, &ax0, &ax1, &ay0, &ay1);
  span(B, &bx0, &bx1, &by0, &by1);
  bool ox = false, oy = false;
  for (long long s : {-NX, 0LL, NX})
    if (ax0 <= bx1 + s && bx0 + s <= ax1) ox = true;
  for (long long s : {-NY, 0LL, NY})
    if (ay0 <= by1 + s && by0 + s <= ay1) oy = true;
  return ox && oy;
}

// Relation of a leaf's side to the region beyond it: 0 same level leaf,
// -1 covered by a coarser leaf, +1 subdivided into finer leaves.
int side_relation(const Hier& h, const Leaf& L, int side) {
  int px = L.ix, py = L.iy;
  if (side == S_W) px -= 1;
  if (side == S_E) px += 1;
  if (side == S_S) py -= 1;
  if (side == S_N) py += 1;
  if (h.find(L.level, px, py) >= 0) return 0;
  if (L.level > 0) {
    const int nx = h.npx(L.level), ny = h.npy(L.level);
    const int wx = ((px % nx) + nx) % nx, wy = ((py % ny) + ny) % ny;
    if (h.find(L.level - 1, wx >> 1, wy >> 1) >= 0) return -1;
  }
  return +1;
}

// ----- Ghost fill (Sec. 3.1, Sec. 3.2) -------------------------------------
//
// The fill set of a patch is every DOF of its block except the averages of
// its interior cells and the nodes strictly inside its interior square.  For
// each such DOF the source is:
//  * averages: the leaf covering the cell -- same level: copy; finer: mean of
//    the four fine averages (fine->coarse transfer); coarser: Simpson 3x3 of
//    the coarse reconstruction over the fine cell (coarse->fine transfer);
//  * nodes: the finest leaf whose closed square contains the node ("fine
//    wins" on coarse-fine lines, matching "point values are copied from the
//    vertices of the fine grid cells"); same or finer: copy the vertex;
//    coarser: evaluate the coarse reconstruction at the node.
// Candidates at one level are tried in the order (hi,hi), (lo,hi), (hi,lo),
// (lo,lo), where hi is the patch containing the position's upper-right side.
// Only leaves of level >= src_min may serve as sources (at a non-synchronised
// time, levels below src_min are at another time level); a DOF without an
// admissible source keeps its value.  Phase A does all same-level and
// fine->coarse transfers, phase B all coarse->fine interpolations (which read
// coarse nodes already corrected in phase A).

bool in_fill_set(const Hier& h, int kind, int i, int j) {
  const int m = h.m;
  if (kind == K_AVG) return !(i >= 0 && i < m && j >= 0 && j < m);
  if (kind == K_CORNER) return !(i >= 1 && i <= m - 1 && j >= 1 && j <= m - 1);
  if (kind == K_XEDGE) return !(i >= 1 && i <= m - 1 && j >= 0 && j <= m - 1);
  return !(i >= 0 && i <= m - 1 && j >= 1 && j <= m - 1);
}

struct Source {
  int leaf = -1;
  int rel = 0;          // level(source) - level(target)
  long long X = 0, Y = 0;  // position in source-level half-cell units, local to the source patch (rel >= 0)
  double xs = 0, ys = 0;   // position in source-level half-cell units, local (rel < 0)
};

long long floordiv(long long a, long long b) {
  long long q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return q;
}

// Node source lookup.  (HX,HY): node position in target-level half-cell
// units (global, unwrapped).
Source node_source(const Hier& h, int lt, long long HX, long long HY, int src_min) {
  Source s;
  // work in level (lt+1) half-cell units
  const long long FX = 2 * HX, FY = 2 * HY;
  for (int k = lt + 1; k >= lt - 1; --k) {
    if (k < 0 || k > h.lmax || k < src_min) continue;
    const int sh = lt + 1 - k;  // level-k half unit = 2^sh fine units
    const long long unit = 1LL << sh;
    const long long P = 2LL * h.m * unit;  // patch size in fine units
    const long long hx = floordiv(FX, P), hy = floordiv(FY, P);
    const bool bx = (FX % P + P) % P == 0, by = (FY % P + P) % P == 0;
    const long long cx[2] = {hx, hx - 1}, cy[2] = {hy, hy - 1};
    const int order[4][2] = {{0, 0}, {1, 0}, {0, 1}, {1, 1}};
    for (const auto& o : order) {
      if (o[0] == 1 && !bx) continue;
      if (o[1] == 1 && !by) continue;
      const int id = h.find(k, int(cx[o[0]]), int(cy[o[1]]));
      if (id < 0) continue;
      s.leaf = id;
      s.rel = k - lt;
      if (k >= lt) {
        s.X = (FX - cx[o[0]] * P) / unit;
        s.Y = (FY - cy[o[1]] * P) / unit;
      } else {
        s.xs = double(FX - cx[o[0]] * P) / double(unit);
        s.ys = double(FY - cy[o[1]] * P) / double(unit);
      }
      return s;
    }
  }
  return s;
}

// Evaluate the reconstruction of a leaf at a local position given in its own
// half-cell units (0..2m along each axis).
double eval_leaf(const Hier& h, const Leaf& L, int comp, double xs, double ys) {
  int ci = int(std::floor(xs / 2.0)), cj = int(std::floor(ys / 2.0));
  ci = std::min(std::max(ci, 0), h.m - 1);
  cj = std::min(std::max(cj, 0), h.m - 1);
  const double xi = xs - (2.0 * ci + 1.0), eta = ys - (2.0 * cj + 1.0);
  BlockGrid bg = h.view(L);
  return cell_eval(bg.cell(comp, ci, cj), xi, eta);
}

// Value of a node of a same-or-finer source at integer local half-unit
// position (X,Y) (both even -> corner, even/odd -> xedge, odd/even -> yedge).
double node_value(const Hier& h, const Leaf& L, int comp, long long X, long long Y) {
  const bool ex = (X % 2) == 0, ey = (Y % 2) == 0;
  if (ex && ey) return h.at(L, K_CORNER, comp, int(X / 2), int(Y / 2));
  if (ex && !ey) return h.at(L, K_XEDGE, comp, int(X / 2), int((Y - 1) / 2));
  if (!ex && ey) return h.at(L, K_YEDGE, comp, int((X - 1) / 2), int(Y / 2));
  die("node lookup hit a cell centre");
}

// Fill, for all target leaves of level >= tmin, with sources of level >= smin.
void fill(Hier& h, int tmin, int smin) {
  const int m = h.m, g = h.g;
  for (int phase = 0; phase < 2; ++phase) {
    for (int t = 0; t < int(h.leaves.size()); ++t) {
      Leaf& T = h.leaves[t];
      const int lt = T.level;
      if (lt < tmin) continue;
      for (int kind = 0; kind < 4; ++kind) {
        const int ihi = (kind == K_AVG || kind == K_YEDGE) ? m + g - 1 : m + g;
        const int jhi = (kind == K_AVG || kind == K_XEDGE) ? m + g - 1 : m + g;
        for (int j = -g; j <= jhi; ++j)
          for (int i = -g; i <= ihi; ++i) {
            if (!in_fill_set(h, kind, i, j)) continue;
            const long long I = (long long)T.ix * m + i, J = (long long)T.iy * m + j;
            if (kind == K_AVG) {
              // covering leaf: same level, then finer, then coarser
              int id = -1, rel = 0;
              const long long px = floordiv(I, m), py = floordiv(J, m);
              if (lt >= smin && (id = h.find(lt, int(px), int(py))) >= 0) rel = 0;
              else if (lt + 1 <= h.lmax && lt + 1 >= smin &&
                       (id = h.find(lt + 1, int(floordiv(2 * I, m)), int(floordiv(2 * J, m)))) >= 0) rel = 1;
              else if (lt - 1 >= 0 && lt - 1 >= smin &&
                       (id = h.find(lt - 1, int(floordiv(I, 2 * m)), int(floordiv(J, 2 * m)))) >= 0) rel = -1;
              if (id < 0) continue;
              if ((phase == 0) != (rel >= 0)) continue;
              const Leaf& Sx = h.leaves[id];
              for (int c = 0; c < h.ncomp; ++c) {
                double val;
                if (rel == 0) {
                  const long long li = I - floordiv(I, m) * m, lj = J - floordiv(J, m) * m;
                  val = h.at(Sx, K_AVG, c, int(li), int(lj));
                } else if (rel == 1) {
                  const long long fi = 2 * I - floordiv(2 * I, m) * m, fj = 2 * J - floordiv(2 * J, m) * m;
                  val = 0.25 * (h.at(Sx, K_AVG, c, int(fi), int(fj)) + h.at(Sx, K_AVG, c, int(fi + 1), int(fj)) +
                                h.at(Sx, K_AVG, c, int(fi), int(fj + 1)) +
                                h.at(Sx, K_AVG, c, int(fi + 1), int(fj + 1)));
                } else {
                  // fine cell (I,J) inside coarse cell (I>>1, J>>1); Simpson 3x3
                  const long long CI = floordiv(I, 2), CJ = floordiv(J, 2);
                  const long long ci = CI - floordiv(CI, m) * m, cj = CJ - floordiv(CJ, m) * m;
                  BlockGrid bg = h.view(Sx);
                  const Cell cc = bg.cell(c, int(ci), int(cj));
                  const double xa = (I - 2 * CI == 0) ? -1.0 : 0.0;
                  const double ya = (J - 2 * CJ == 0) ? -1.0 : 0.0;
                  const double w[3] = {1.0, 4.0, 1.0};
                  double sum = 0.0;
                  for (int p = 0; p < 3; ++p)
                    for (int q = 0; q < 3; ++q)
                      sum += w[p] * w[q] * cell_eval(cc, xa + 0.5 * p, ya + 0.5 * q);
                  val = sum / 36.0;
                }
                h.at(T, K_AVG, c, i, j) = val;
              }
            } else {
              long long HX = 2 * I, HY = 2 * J;
              if (kind == K_XEDGE) HY += 1;
              if (kind == K_YEDGE) HX += 1;
              const Source s = node_source(h, lt, HX, HY, smin);
              if (s.leaf < 0) continue;
              if ((phase == 0) != (s.rel >= 0)) continue;
              // the target itself at the same position is the finest: keep;
              // a periodic image of the node inside the target is a source
              if (s.leaf == t && s.rel == 0 && s.X == HX - 2LL * m * T.ix && s.Y == HY - 2LL * m * T.iy)
                continue;
              const Leaf& Sx = h.leaves[s.leaf];
              for (int c = 0; c < h.ncomp; ++c) {
                const double val = (s.rel >= 0) ? node_value(h, Sx, c, s.X, s.Y)
                                                : eval_leaf(h, Sx, c, s.xs, s.ys);
                h.at(T, kind, c, i, j) = val;
              }
            }
          }
      }
    }
  }
}

// ----- One level substep -----------------------------------------------------
// region 0: interior cells [0,m); region 1: interior plus ghost layer 1,
// cells [-1,m+1).  Writes new averages of the region and new point values of
// all nodes on the boundaries of its cells.  For every side whose neighbour
// is at another level, adds F * (face length) * dt of each boundary face of
// the interior block to the leaf's flux register.
void step_leaf(Hier& h, Leaf& L, double dt, int region) {
  BlockGrid bg = h.view(L);
  const int lo = region ? -1 : 0, hi = region ? h.m + 1 : h.m;
  const StepResult r = af_step_range(bg, h.ph, dt, lo, hi, lo, hi);
  const int nc = h.ncomp, NI = r.ni + 1;
  std::vector<double> nb[4];
  for (int k = 0; k < 4; ++k) nb[k] = L.blk[k];
  for (int j = lo; j < hi; ++j)
    for (int i = lo; i < hi; ++i)
      for (int c = 0; c < nc; ++c)
        nb[K_AVG][h.bidx(c, i, j)] = r.avg[(size_t(j - lo) * r.ni + size_t(i - lo)) * nc + c];
  for (int j = lo; j <= hi; ++j)
    for (int i = lo; i <= hi; ++i)
      for (int c = 0; c < nc; ++c) {
        const size_t s = (size_t(j - lo) * NI + size_t(i - lo)) * nc + c;
        nb[K_CORNER][h.bidx(c, i, j)] = r.corner[s];
        if (j < hi) nb[K_XEDGE][h.bidx(c, i, j)] = r.xedge[s];
        if (i < hi) nb[K_YEDGE][h.bidx(c, i, j)] = r.yedge[s];
      }
  // flux registers on the boundary of the interior block
  const int m = h.m;
  for (int side = 0; side < 4; ++side) {
    if (side_relation(h, L, side) == 0) continue;
    for (int k = 0; k < m; ++k)
      for (int c = 0; c < nc; ++c) {
        double F;
        if (side == S_W || side == S_E) {
          const int i = (side == S_W) ? 0 : m;
          F = r.Fx[(size_t(k - lo) * NI + size_t(i - lo)) * nc + c] * bg.dy * dt;
        } else {
          const int j = (side == S_S) ? 0 : m;
          F = r.Gy[(size_t(j - lo) * r.ni + size_t(k - lo)) * nc + c] * bg.dx * dt;
        }
        L.reg[(size_t(side) * m + k) * nc + c] += F;
      }
  }
  for (int k = 0; k < 4; ++k) L.blk[k] = nb[k];
}

void step_level(Hier& h, int l, double t, double dt, int region) {
  h.ph.t = t;
  for (Leaf& L : h.leaves)
    if (L.level == l) step_leaf(h, L, dt, region);
}

// ----- Conservative fix (Sec. 3.2, Berger-Colella) --------------------------
// For each coarse leaf of level l and each side facing finer leaves, replace
// the coarse flux contribution by the sum of the fine ones:
//   Q_c += s (Fc*len_c*dt_c - sum Ff*len_f*dt_f) / (dx_c dy_c),  s = +1 on the
// east/north side, -1 on the west/south side.  Registers used are cleared.
void flux_correct(Hier& h, int l) {
  const int m = h.m, nc = h.ncomp;
  for (Leaf& C : h.leaves) {
    if (C.level != l) continue;
    const double area = h.dx(l) * h.dy(l);
    for (int side = 0; side < 4; ++side) {
      if (side_relation(h, C, side) != 1) continue;
      const int opp = side ^ 1;
      for (int k = 0; k < m; ++k) {
        // fine cells 2K, 2K+1 along the side (global level l+1 index)
        const long long K = (side == S_W || side == S_E) ? (long long)C.iy * m + k
                                                          : (long long)C.ix * m + k;
        const long long f0 = 2 * K;
        int fpx, fpy;
        if (side == S_W || side == S_E) {
          fpx = (side == S_W) ? 2 * C.ix - 1 : 2 * C.ix + 2;
          fpy = int(floordiv(f0, m));
        } else {
          fpy = (side == S_S) ? 2 * C.iy - 1 : 2 * C.iy + 2;
          fpx = int(floordiv(f0, m));
        }
        const int fid = h.find(l + 1, fpx, fpy);
        if (fid < 0) die("flux_correct: missing fine leaf");
        const Leaf& F = h.leaves[fid];
        const int fk = int(f0 - floordiv(f0, m) * m);
        const int ci = (side == S_W) ? 0 : (side == S_E ? m - 1 : k);
        const int cj = (side == S_S) ? 0 : (side == S_N ? m - 1 : k);
        const double sgn = (side == S_E || side == S_N) ? 1.0 : -1.0;
        for (int c = 0; c < nc; ++c) {
          const double rc = C.reg[(size_t(side) * m + k) * nc + c];
          const double rf = F.reg[(size_t(opp) * m + fk) * nc + c] +
                            F.reg[(size_t(opp) * m + fk + 1) * nc + c];
          h.at(C, K_AVG, c, ci, cj) += sgn * (rc - rf) / area;
        }
      }
    }
  }
  // clear registers of level l (coarse side) and level l+1 sides facing coarser
  for (Leaf& L : h.leaves) {
    if (L.level == l) {
      for (int side = 0; side < 4; ++side)
        if (side_relation(h, L, side) == 1)
          std::fill(L.reg.begin() + size_t(side) * m * nc, L.reg.begin() + size_t(side + 1) * m * nc, 0.0);
    } else if (L.level == l + 1) {
      for (int side = 0; side < 4; ++side)
        if (side_relation(h, L, side) == -1)
          std::fill(L.reg.begin() + size_t(side) * m * nc, L.reg.begin() + size_t(side + 1) * m * nc, 0.0);
    }
  }
}

// ----- Subcycling (Sec. 3.2) ------------------------------------------------
// Level l+1 takes two steps of dt_l/2 per step of level l; cross-level ghost
// data is exchanged only at synchronised times (no time interpolation); the
// first step of each pair also advances ghost layer 1, which supplies the
// ghost data over coarser patches for the second step.
int finest_level(const Hier& h) {
  int f = 0;
  for (const Leaf& L : h.leaves) f = std::max(f, L.level);
  return f;
}

void advance(Hier& h, int l, double t, double dt, bool first, int lfin) {
  step_level(h, l, t, dt, (l > 0 && first) ? 1 : 0);
  if (l + 1 <= lfin) {
    advance(h, l + 1, t, 0.5 * dt, true, lfin);
    fill(h, l + 1, l + 1);
    advance(h, l + 1, t + 0.5 * dt, 0.5 * dt, false, lfin);
    flux_correct(h, l);
  }
}

void coarse_step(Hier& h, double dt0) {
  fill(h, 0, 0);
  advance(h, 0, h.time, dt0, true, finest_level(h));
  h.time += dt0;
}

// Global time stepping (no subcycling, the corollary of Sec. 4.3): every
// level takes one step dt from the same synchronised state, then each coarse
// level's fluxes at finer neighbours are replaced by the fine ones.
void global_step(Hier& h, double dt) {
  fill(h, 0, 0);
  const int lfin = finest_level(h);
  for (int l = 0; l <= lfin; ++l) step_level(h, l, h.time, dt, 0);
  for (int l = 0; l < lfin; ++l) flux_correct(h, l);
  h.time += dt;
}

// ----- Transfers (Sec. 3.1) -------------------------------------------------

// coarse -> fine: child (qx,qy) of coarse leaf C; fills the child's interior
// averages (Simpson 3x3 over each fine cell) and every node of its closed
// square (evaluation of the coarse reconstruction).
void refine_into(const Hier& h, const Leaf& C, int qx, int qy, Leaf& F) {
  const int m = h.m;
  BlockGrid bg = h.view(C);
  for (int c = 0; c < h.ncomp; ++c) {
    for (int j = 0; j < m; ++j)
      for (int i = 0; i < m; ++i) {
        const int fi = qx * m + i, fj = qy * m + j;  // fine index within the parent
        const Cell cc = bg.cell(c, fi / 2, fj / 2);
        const double xa = (fi % 2 == 0) ? -1.0 : 0.0, ya = (fj % 2 == 0) ? -1.0 : 0.0;
        const double w[3] = {1.0, 4.0, 1.0};
        double sum = 0.0;
        for (int p = 0; p < 3; ++p)
          for (int q = 0; q < 3; ++q) sum += w[p] * w[q] * cell_eval(cc, xa + 0.5 * p, ya + 0.5 * q);
        F.blk[K_AVG][h.bidx(c, i, j)] = sum / 36.0;
      }
    for (int j = 0; j <= m; ++j)
      for (int i = 0; i <= m; ++i)
        for (int kind = 1; kind < 4; ++kind) {
          if (kind == K_XEDGE && j == m) continue;
          if (kind == K_YEDGE && i == m) continue;
          // fine-level half units within the parent
          double hx = 2.0 * (qx * m + i), hy = 2.0 * (qy * m + j);
          if (kind == K_XEDGE) hy += 1.0;
          if (kind == K_YEDGE) hx += 1.0;
          F.blk[kind][h.bidx(c, i, j)] = eval_leaf(h, C, c, 0.5 * hx, 0.5 * hy);
        }
  }
}

// fine -> coarse: averages are the mean of four fine averages, nodes are
// copied from the fine vertices (first child containing the node, in the
// candidate order (hi,hi), (lo,hi), (hi,lo), (lo,lo)).
void coarsen_into(const Hier& h, const Leaf* kids[2][2], Leaf& C) {
  const int m = h.m;
  for (int c = 0; c < h.ncomp; ++c) {
    for (int j = 0; j < m; ++j)
      for (int i = 0; i < m; ++i) {
        const int fi = 2 * i, fj = 2 * j;
        const Leaf& K = *kids[fj / m][fi / m];
        const int li = fi % m, lj = fj % m;
        C.blk[K_AVG][h.bidx(c, i, j)] =
            0.25 * (h.at(K, K_AVG, c, li, lj) + h.at(K, K_AVG, c, li + 1, lj) +
                    h.at(K, K_AVG, c, li, lj + 1) + h.at(K, K_AVG, c, li + 1, lj + 1));
      }
    for (int j = 0; j <= m; ++j)
      for (int i = 0; i <= m; ++i)
        for (int kind = 1; kind < 4; ++kind) {
          if (kind == K_XEDGE && j == m) continue;
          if (kind == K_YEDGE && i == m) continue;
          int FX = 2 * i, FY = 2 * j;  // fine corner index within the parent
          if (kind == K_XEDGE) FY += 1;
          if (kind == K_YEDGE) FX += 1;
          // child containing the fine corner (FX,FY), hi candidate first
          int qx = std::min(FX / m, 1), qy = std::min(FY / m, 1);
          C.blk[kind][h.bidx(c, i, j)] = h.at(*kids[qy][qx], K_CORNER, c, FX - qx * m, FY - qy * m);
        }
  }
}

// ----- Tagging (Sec. 3 and Sec. 4.1 / 4.4 / 4.5 criteria) -------------------
// mode 0: max centred gradient of averages over interior cells (uses ghost
// layer 1); mode 1: max - min of interior averages.  Refine if value >= theta_r
// and level < lmax; coarsen-candidate if value < theta_c and level > 0.
int tag_leaf(const Hier& h, const Leaf& L, int mode, int comp, double tr, double tc,
             double* value) {
  const int m = h.m;
  double v;
  if (mode == 0) {
    v = 0.0;
    const double dx = h.dx(L.level), dy = h.dy(L.level);
    for (int j = 0; j < m; ++j)
      for (int i = 0; i < m; ++i) {
        const double gx = std::fabs(h.at(L, K_AVG, comp, i + 1, j) - h.at(L, K_AVG, comp, i - 1, j)) / (2.0 * dx);
        const double gy = std::fabs(h.at(L, K_AVG, comp, i, j + 1) - h.at(L, K_AVG, comp, i, j - 1)) / (2.0 * dy);
        v = std::max(v, std::max(gx, gy));
      }
  } else {
    double lo = h.at(L, K_AVG, comp, 0, 0), hi = lo;
    for (int j = 0; j < m; ++j)
      for (int i = 0; i < m; ++i) {
        lo = std::min(lo, h.at(L, K_AVG, comp, i, j));
        hi = std::max(hi, h.at(L, K_AVG, comp, i, j));
      }
    v = hi - lo;
  }
  if (value) *value = v;
  if (v >= tr && L.level < h.lmax) return 1;
  if (v < tc && L.level > 0) return -1;
  return 0;
}

// ----- Regrid (Sec. 3: refine, family coarsening, 2:1 balance) -------------
// (a) refine every leaf tagged +1 (level < lmax);
// (b) balance closure: while some leaf touches (edge or corner, periodic) a
//     leaf two or more levels finer, refine it;
// (c) a family of four sibling leaves coarsens if all four are tagged -1 and
//     the parent would touch no leaf finer than the siblings; all qualifying
//     families are judged on the set after (b) and coarsen together;
// (d) DOFs are transferred (Sec. 3.1), leaves are sorted by (level, iy, ix),
//     flux registers cleared, and a full ghost fill follows.
struct Key {
  int l, x, y;
  bool operator<(const Key& o) const { return std::tie(l, y, x) < std::tie(o.l, o.y, o.x); }
};

void regrid(Hier& h, const int8_t* tags) {
  const int n = int(h.leaves.size());
  // (a) + (b) on the key set; remember provenance
  std::map<Key, int> tagof;
  for (int k = 0; k < n; ++k) tagof[{h.leaves[k].level, h.leaves[k].ix, h.leaves[k].iy}] = tags[k];
  std::vector<Key> cur;
  for (int k = 0; k < n; ++k) {
    const Leaf& L = h.leaves[k];
    if (tags[k] == 1 && L.level < h.lmax) {
      for (int q = 0; q < 4; ++q) cur.push_back({L.level + 1, 2 * L.ix + (q & 1), 2 * L.iy + (q >> 1)});
    } else {
      cur.push_back({L.level, L.ix, L.iy});
    }
  }
  auto as_leaf = [](const Key& k) { Leaf L; L.level = k.l; L.ix = k.x; L.iy = k.y; return L; };
  const int lref = h.lmax;
  for (;;) {
    bool changed = false;
    std::vector<Key> next;
    for (size_t a = 0; a < cur.size(); ++a) {
      bool split = false;
      const Leaf A = as_leaf(cur[a]);
      for (size_t b = 0; b < cur.size() && !split; ++b) {
        if (cur[b].l < cur[a].l + 2) continue;
        if (touches(h, A, as_leaf(cur[b]), lref)) split = true;
      }
      if (split) {
        changed = true;
        for (int q = 0; q < 4; ++q) next.push_back({A.level + 1, 2 * A.ix + (q & 1), 2 * A.iy + (q >> 1)});
      } else {
        next.push_back(cur[a]);
      }
    }
    cur.swap(next);
    if (!changed) break;
  }
  // (c) families
  std::map<Key, int> present;
  for (size_t a = 0; a < cur.size(); ++a) present[cur[a]] = int(a);
  std::vector<char> drop(cur.size(), 0);
  std::vector<Key> parents;
  for (size_t a = 0; a < cur.size(); ++a) {
    const Key k = cur[a];
    if (k.l == 0 || (k.x & 1) || (k.y & 1)) continue;  // visit each family via its (even,even) child
    bool all = true;
    int idx[4];
    for (int q = 0; q < 4; ++q) {
      const Key s{k.l, k.x + (q & 1), k.y + (q >> 1)};
      auto it = present.find(s);
      auto tg = tagof.find(s);
      if (it == present.end() || tg == tagof.end() || tg->second != -1) { all = false; break; }
      idx[q] = it->second;
    }
    if (!all) continue;
    const Leaf P = as_leaf({k.l - 1, k.x >> 1, k.y >> 1});
    bool ok = true;
    for (size_t b = 0; b < cur.size() && ok; ++b)
      if (cur[b].l > k.l && touches(h, P, as_leaf(cur[b]), lref)) ok = false;
    if (!ok) continue;
    for (int q = 0; q < 4; ++q) drop[idx[q]] = 1;
    parents.push_back({k.l - 1, k.x >> 1, k.y >> 1});
  }
  std::vector<Key> fin;
  for (size_t a = 0; a < cur.size(); ++a)
    if (!drop[a]) fin.push_back(cur[a]);
  for (const Key& p : parents) fin.push_back(p);
  std::sort(fin.begin(), fin.end());
  // (d) transfers
  std::vector<Leaf> out(fin.size());
  for (size_t a = 0; a < fin.size(); ++a) {
    Leaf& L = out[a];
    L.level = fin[a].l; L.ix = fin[a].x; L.iy = fin[a].y;
    h.alloc(L);
    const int same = h.find(L.level, L.ix, L.iy);
    if (same >= 0) {
      for (int k = 0; k < 4; ++k) L.blk[k] = h.leaves[same].blk[k];
      continue;
    }
    // an ancestor that is an old leaf: refine down level by level
    int anc_level = -1, anc = -1;
    for (int l = L.level - 1; l >= 0; --l) {
      const int id = h.find(l, L.ix >> (L.level - l), L.iy >> (L.level - l));
      if (id >= 0) { anc_level = l; anc = id; break; }
    }
    if (anc >= 0) {
      Leaf tmp = h.leaves[anc];
      for (int l = anc_level; l < L.level; ++l) {
        const int sh = L.level - l - 1;
        const int qx = (L.ix >> sh) & 1, qy = (L.iy >> sh) & 1;
        Leaf child;
        child.level = l + 1; child.ix = L.ix >> sh; child.iy = L.iy >> sh;
        h.alloc(child);
        refine_into(h, tmp, qx, qy, child);
        tmp = child;
      }
      for (int k = 0; k < 4; ++k) L.blk[k] = tmp.blk[k];
      continue;
    }
    // otherwise: four old children
    const Leaf* kids[2][2];
    for (int q = 0; q < 4; ++q) {
      const int id = h.find(L.level + 1, 2 * L.ix + (q & 1), 2 * L.iy + (q >> 1));
      if (id < 0) die("regrid: coarsened family incomplete");
      kids[q >> 1][q & 1] = &h.leaves[id];
    }
    coarsen_into(h, kids, L);
  }
  h.leaves.swap(out);
  h.reindex();
  fill(h, 0, 0);
}

}  // namespace

// ===========================================================================
// C interface (ctypes).
// ===========================================================================
extern "C" {

// --- elementary pieces (for pins) -------------------------------------------

// Evaluate the reconstruction of one cell at reference points.
// dofs = [avg, c_ll, c_rl, c_lu, c_ru, e_l, e_r, e_b, e_t]
void or_recon_eval(const double* dofs, int n, const double* xi, const double* eta, double* out) {
  const Cell c = make_cell(dofs[0], dofs[1], dofs[2], dofs[3], dofs[4], dofs[5], dofs[6], dofs[7], dofs[8]);
  for (int k = 0; k < n; ++k) out[k] = cell_eval(c, xi[k], eta[k]);
}

// Quarter-disc spherical mean of zx^m zy^n (coefficient grid 4x4).
double or_sector_mean(const double* coef16, int quad, double R, double* r_dmean) {
  double c4[4][4];
  for (int m = 0; m < 4; ++m)
    for (int n = 0; n < 4; ++n) c4[m][n] = coef16[m * 4 + n];
  double M, dM;
  sector_mean(c4, quad, R, &M, &dM);
  if (r_dmean) *r_dmean = dM;
  return M;
}

// --- periodic single grid ---------------------------------------------------
}  // extern "C"

namespace {

// One AF step on a periodic grid in place; arrays [ncomp][ny][nx].
void step_periodic(const Physics& ph, int nx, int ny, double x0, double y0, double dx, double dy,
                   double dt, double* avg, double* corner, double* xedge, double* yedge) {
  PeriodicGrid pg;
  pg.nx = nx; pg.ny = ny; pg.dx = dx; pg.dy = dy; pg.ox = x0; pg.oy = y0;
  pg.ncomp = ph.eq == 1 ? 3 : 1;
  pg.arr[K_AVG] = avg; pg.arr[K_CORNER] = corner; pg.arr[K_XEDGE] = xedge; pg.arr[K_YEDGE] = yedge;
  const StepResult r = af_step_range(pg, ph, dt, 0, nx, 0, ny);
  const int nc = pg.ncomp, NI = nx + 1;
  std::vector<double> na(size_t(nc) * nx * ny), nco(na.size()), nxe(na.size()), nye(na.size());
  for (int comp = 0; comp < nc; ++comp)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const size_t d = (size_t(comp) * ny + j) * nx + i;
        na[d] = r.avg[(size_t(j) * nx + i) * nc + comp];
        const size_t s = (size_t(j) * NI + i) * nc + comp;
        nco[d] = r.corner[s];
        nxe[d] = r.xedge[s];
        nye[d] = r.yedge[s];
      }
  std::memcpy(avg, na.data(), na.size() * sizeof(double));
  std::memcpy(corner, nco.data(), na.size() * sizeof(double));
  std::memcpy(xedge, nxe.data(), na.size() * sizeof(double));
  std::memcpy(yedge, nye.data(), na.size() * sizeof(double));
}

// One step of one patch block; see or_patch_step.
void patch_step(const Physics& ph, int m, int g, double x0p, double y0p, double dx, double dy,
                double dt, int region, const double* in_avg, const double* in_corner,
                const double* in_xedge, const double* in_yedge, double* out_avg, double* out_corner,
                double* out_xedge, double* out_yedge, double* flux4, int side_mask) {
  BlockGrid bg;
  bg.m = m; bg.g = g; bg.dx = dx; bg.dy = dy; bg.ox = x0p; bg.oy = y0p;
  bg.ncomp = ph.eq == 1 ? 3 : 1;
  bg.arr[K_AVG] = in_avg; bg.arr[K_CORNER] = in_corner; bg.arr[K_XEDGE] = in_xedge; bg.arr[K_YEDGE] = in_yedge;
  const int lo = region ? -1 : 0, hi = region ? m + 1 : m;
  const StepResult r = af_step_range(bg, ph, dt, lo, hi, lo, hi);
  const int nc = bg.ncomp, NI = r.ni + 1;
  const size_t pl = bg.plane();
  std::memcpy(out_avg, in_avg, pl * nc * sizeof(double));
  std::memcpy(out_corner, in_corner, pl * nc * sizeof(double));
  std::memcpy(out_xedge, in_xedge, pl * nc * sizeof(double));
  std::memcpy(out_yedge, in_yedge, pl * nc * sizeof(double));
  for (int comp = 0; comp < nc; ++comp) {
    for (int j = lo; j < hi; ++j)
      for (int i = lo; i < hi; ++i)
        out_avg[bg.idx(comp, i, j)] = r.avg[(size_t(j - lo) * r.ni + size_t(i - lo)) * nc + comp];
    for (int j = lo; j <= hi; ++j)
      for (int i = lo; i <= hi; ++i) {
        const size_t s = (size_t(j - lo) * NI + size_t(i - lo)) * nc + comp;
        out_corner[bg.idx(comp, i, j)] = r.corner[s];
        if (j < hi) out_xedge[bg.idx(comp, i, j)] = r.xedge[s];
        if (i < hi) out_yedge[bg.idx(comp, i, j)] = r.yedge[s];
      }
  }
  if (flux4) {
    for (int side = 0; side < 4; ++side) {
      if (!(side_mask & (1 << side))) continue;
      for (int k = 0; k < m; ++k)
        for (int comp = 0; comp < nc; ++comp) {
          double F;
          if (side < 2) {
            const int i = side == 0 ? 0 : m;
            F = r.Fx[(size_t(k - lo) * NI + size_t(i - lo)) * nc + comp] * dy * dt;
          } else {
            const int j = side == 2 ? 0 : m;
            F = r.Gy[(size_t(j - lo) * r.ni + size_t(k - lo)) * nc + comp] * dx * dt;
          }
          flux4[(size_t(side) * m + k) * nc + comp] += F;
        }
    }
  }
}

Physics physics(int eq, double a, double b, double c) {
  Physics ph;
  ph.eq = eq; ph.a = a; ph.b = b; ph.c = c;
  return ph;
}

Physics rotation(double omega, double xc, double yc) {
  Physics ph;
  ph.eq = 2; ph.omega = omega; ph.xc = xc; ph.yc = yc;
  return ph;
}

}  // namespace

extern "C" {

// One AF step on a periodic nx x ny grid, in place.  Arrays [ncomp][ny][nx].
// eq 0 advection (a, b), 1 acoustics (c), 4 Burgers.
void or_step_periodic(int eq, int nx, int ny, double dx, double dy, double dt, double a,
                      double b, double c, double* avg, double* corner, double* xedge,
                      double* yedge) {
  step_periodic(physics(eq, a, b, c), nx, ny, 0.0, 0.0, dx, dy, dt, avg, corner, xedge, yedge);
}

// Several steps on the periodic grid (saves ctypes round trips).
void or_run_periodic(int eq, int nx, int ny, double dx, double dy, double dt, int nsteps,
                     double a, double b, double c, double* avg, double* corner, double* xedge,
                     double* yedge) {
  const Physics ph = physics(eq, a, b, c);
  for (int s = 0; s < nsteps; ++s) step_periodic(ph, nx, ny, 0.0, 0.0, dx, dy, dt, avg, corner, xedge, yedge);
}

// Solid-body rotation a = -omega (y - yc), b = omega (x - xc) on the periodic
// grid whose cell (0,0) has its lower-left corner at (x0, y0) (Sec. 4.2).
void or_run_periodic_rot(int nx, int ny, double x0, double y0, double dx, double dy, double dt,
                         int nsteps, double omega, double xc, double yc, double* avg,
                         double* corner, double* xedge, double* yedge) {
  const Physics ph = rotation(omega, xc, yc);
  for (int s = 0; s < nsteps; ++s) step_periodic(ph, nx, ny, x0, y0, dx, dy, dt, avg, corner, xedge, yedge);
}

// Swirl flow (Sec. 4.3) on the periodic grid, starting at time t0.
void or_run_periodic_swirl(int nx, int ny, double x0, double y0, double dx, double dy, double dt,
                           int nsteps, double t0, double* avg, double* corner, double* xedge,
                           double* yedge) {
  Physics ph;
  ph.eq = 3;
  for (int s = 0; s < nsteps; ++s) {
    ph.t = t0 + s * dt;
    step_periodic(ph, nx, ny, x0, y0, dx, dy, dt, avg, corner, xedge, yedge);
  }
}

// --- one patch block --------------------------------------------------------
// blocks: four arrays [ncomp][(m+2g+1)^2], row-major (row = j+g, col = i+g).
// region 0 = interior, 1 = interior + ghost layer 1.  `out` receives the
// updated averages of the region's cells and the new values of all nodes on
// their boundaries (other entries are copied from `in`).  flux4 (may be NULL)
// receives F * face-length * dt on the four sides of the interior block,
// [side W,E,S,N][m][ncomp], accumulated (+=) for sides whose bit is set in
// side_mask.
void or_patch_step(int eq, int m, int g, double dx, double dy, double dt, double a, double b,
                   double c, int region, const double* in_avg, const double* in_corner,
                   const double* in_xedge, const double* in_yedge, double* out_avg,
                   double* out_corner, double* out_xedge, double* out_yedge, double* flux4,
                   int side_mask) {
  patch_step(physics(eq, a, b, c), m, g, 0.0, 0.0, dx, dy, dt, region, in_avg, in_corner, in_xedge,
             in_yedge, out_avg, out_corner, out_xedge, out_yedge, flux4, side_mask);
}

// The same for solid-body rotation; (x0p, y0p) is the lower-left corner of
// the patch's cell (0,0).
void or_patch_step_rot(int m, int g, double x0p, double y0p, double dx, double dy, double dt,
                       double omega, double xc, double yc, int region, const double* in_avg,
                       const double* in_corner, const double* in_xedge, const double* in_yedge,
                       double* out_avg, double* out_corner, double* out_xedge, double* out_yedge,
                       double* flux4, int side_mask) {
  patch_step(rotation(omega, xc, yc), m, g, x0p, y0p, dx, dy, dt, region, in_avg, in_corner, in_xedge,
             in_yedge, out_avg, out_corner, out_xedge, out_yedge, flux4, side_mask);
}

// The same for the swirl flow, the step starting at time t.
void or_patch_step_swirl(int m, int g, double x0p, double y0p, double dx, double dy, double dt,
                         double t, int region, const double* in_avg, const double* in_corner,
                         const double* in_xedge, const double* in_yedge, double* out_avg,
                         double* out_corner, double* out_xedge, double* out_yedge, double* flux4,
                         int side_mask) {
  Physics ph;
  ph.eq = 3;
  ph.t = t;
  patch_step(ph, m, g, x0p, y0p, dx, dy, dt, region, in_avg, in_corner, in_xedge, in_yedge, out_avg,
             out_corner, out_xedge, out_yedge, flux4, side_mask);
}

// Burgers (Sec. 2.2) on one patch block with a given number of fixed-point
// iterations per point value (two in the method; other counts for pins).
void or_patch_step_burgers(int m, int g, double dx, double dy, double dt, int iters, int region,
                           const double* in_avg, const double* in_corner, const double* in_xedge,
                           const double* in_yedge, double* out_avg, double* out_corner, double* out_xedge,
                           double* out_yedge, double* flux4, int side_mask) {
  Physics ph;
  ph.eq = 4;
  ph.iters = iters;
  patch_step(ph, m, g, 0.0, 0.0, dx, dy, dt, region, in_avg, in_corner, in_xedge, in_yedge, out_avg,
             out_corner, out_xedge, out_yedge, flux4, side_mask);
}

// Swirl foot of one node (for pins): the point reached from (x, y) at time
// t + tau by the Runge-Kutta step back to t, on a grid of spacing (dx, dy).
void or_swirl_foot(double x, double y, double t, double tau, double dx, double dy, double* fx, double* fy) {
  PeriodicGrid g;
  g.dx = dx;
  g.dy = dy;
  swirl_trace(g, x, y, t, tau, fx, fy);
}

// --- AMR hierarchy ------------------------------------------------------------
void* or_hier_new(int eq, int m, int n0x, int n0y, int lmax, double x0, double y0, double lx,
                  double ly, double a, double b, double c) {
  Hier* h = new Hier();
  h->ph.eq = eq; h->ph.a = a; h->ph.b = b; h->ph.c = c;
  h->m = m; h->g = 2; h->ncomp = eq == 1 ? 3 : 1;
  h->n0x = n0x; h->n0y = n0y; h->lmax = lmax;
  h->x0 = x0; h->y0 = y0; h->lx = lx; h->ly = ly;
  return h;
}
void or_hier_free(void* hp) { delete static_cast<Hier*>(hp); }

// Switch the hierarchy's equation to the swirl flow of Sec. 4.3.
void or_hier_set_swirl(void* hp) {
  Hier* h = static_cast<Hier*>(hp);
  h->ph = Physics();
  h->ph.eq = 3;
  h->ncomp = 1;
}

// Switch the hierarchy's equation to solid-body rotation about (xc, yc).
void or_hier_set_rotation(void* hp, double omega, double xc, double yc) {
  Hier* h = static_cast<Hier*>(hp);
  h->ph = rotation(omega, xc, yc);
  h->ncomp = 1;
}

// Replace the leaf set (data zeroed).  Leaves are kept in the given order.
void or_hier_set_leaves(void* hp, int n, const int* level, const int* ix, const int* iy) {
  Hier& h = *static_cast<Hier*>(hp);
  h.leaves.assign(n, Leaf());
  for (int k = 0; k < n; ++k) {
    h.leaves[k].level = level[k]; h.leaves[k].ix = ix[k]; h.leaves[k].iy = iy[k];
    h.alloc(h.leaves[k]);
  }
  h.reindex();
}
int or_hier_num_leaves(void* hp) { return int(static_cast<Hier*>(hp)->leaves.size()); }
void or_hier_get_leaves(void* hp, int* level, int* ix, int* iy) {
  Hier& h = *static_cast<Hier*>(hp);
  for (size_t k = 0; k < h.leaves.size(); ++k) {
    level[k] = h.leaves[k].level; ix[k] = h.leaves[k].ix; iy[k] = h.leaves[k].iy;
  }
}
// kind 0..3; data [ncomp][(m+5)^2]
void or_hier_set_block(void* hp, int leaf, int kind, const double* data) {
  Hier& h = *static_cast<Hier*>(hp);
  std::memcpy(h.leaves[leaf].blk[kind].data(), data, h.plane() * h.ncomp * sizeof(double));
}
void or_hier_get_block(void* hp, int leaf, int kind, double* data) {
  Hier& h = *static_cast<Hier*>(hp);
  std::memcpy(data, h.leaves[leaf].blk[kind].data(), h.plane() * h.ncomp * sizeof(double));
}
void or_hier_get_reg(void* hp, int leaf, double* data) {
  Hier& h = *static_cast<Hier*>(hp);
  std::memcpy(data, h.leaves[leaf].reg.data(), h.leaves[leaf].reg.size() * sizeof(double));
}
void or_hier_set_reg(void* hp, int leaf, const double* data) {
  Hier& h = *static_cast<Hier*>(hp);
  std::memcpy(h.leaves[leaf].reg.data(), data, h.leaves[leaf].reg.size() * sizeof(double));
}
// side relations [n][4] : 0 same, -1 coarser, +1 finer
void or_hier_side_relations(void* hp, int* rel) {
  Hier& h = *static_cast<Hier*>(hp);
  for (size_t k = 0; k < h.leaves.size(); ++k)
    for (int s = 0; s < 4; ++s) rel[k * 4 + s] = side_relation(h, h.leaves[k], s);
}
void or_hier_fill(void* hp, int tmin, int smin) { fill(*static_cast<Hier*>(hp), tmin, smin); }
void or_hier_step_level(void* hp, int level, double dt, int region) {
  Hier& h = *static_cast<Hier*>(hp);
  step_level(h, level, h.time, dt, region);
}
void or_hier_flux_correct(void* hp, int level) { flux_correct(*static_cast<Hier*>(hp), level); }
void or_hier_coarse_step(void* hp, double dt0) { coarse_step(*static_cast<Hier*>(hp), dt0); }
void or_hier_run(void* hp, double dt0, int nsteps) {
  for (int s = 0; s < nsteps; ++s) coarse_step(*static_cast<Hier*>(hp), dt0);
}
// Global time stepping (no subcycling): nsteps steps of dt for every level.
void or_hier_run_global(void* hp, double dt, int nsteps) {
  for (int s = 0; s < nsteps; ++s) global_step(*static_cast<Hier*>(hp), dt);
}
void or_hier_set_time(void* hp, double t) { static_cast<Hier*>(hp)->time = t; }
double or_hier_get_time(void* hp) { return static_cast<Hier*>(hp)->time; }
void or_hier_tag(void* hp, int mode, int comp, double tr, double tc, int8_t* tags, double* values) {
  Hier& h = *static_cast<Hier*>(hp);
  for (size_t k = 0; k < h.leaves.size(); ++k)
    tags[k] = int8_t(tag_leaf(h, h.leaves[k], mode, comp, tr, tc, values ? &values[k] : nullptr));
}
void or_hier_regrid(void* hp, const int8_t* tags) { regrid(*static_cast<Hier*>(hp), tags); }
// sum over leaves of interior averages times cell area, per component
void or_hier_sum(void* hp, double* out) {
  Hier& h = *static_cast<Hier*>(hp);
  for (int c = 0; c < h.ncomp; ++c) out[c] = 0.0;
  for (const Leaf& L : h.leaves) {
    const double area = h.dx(L.level) * h.dy(L.level);
    for (int c = 0; c < h.ncomp; ++c)
      for (int j = 0; j < h.m; ++j)
        for (int i = 0; i < h.m; ++i) out[c] += h.at(L, K_AVG, c, i, j) * area;
  }
}
// 1 if every pair of touching leaves differs by at most one level
int or_hier_balanced(void* hp) {
  Hier& h = *static_cast<Hier*>(hp);
  for (size_t a = 0; a < h.leaves.size(); ++a)
    for (size_t b = 0; b < h.leaves.size(); ++b)
      if (h.leaves[b].level >= h.leaves[a].level + 2 &&
          touches(h, h.leaves[a], h.leaves[b], h.lmax))
        return 0;
  return 1;
}
// refine leaf `leaf` data into child (qx,qy), output four block arrays
void or_refine_block(void* hp, int leaf, int qx, int qy, double* out_avg, double* out_corner,
                     double* out_xedge, double* out_yedge) {
  Hier& h = *static_cast<Hier*>(hp);
  Leaf F;
  h.alloc(F);
  refine_into(h, h.leaves[leaf], qx, qy, F);
  double* outs[4] = {out_avg, out_corner, out_xedge, out_yedge};
  for (int k = 0; k < 4; ++k) std::memcpy(outs[k], F.blk[k].data(), F.blk[k].size() * sizeof(double));
}
// coarsen the four leaves kid[qy*2+qx] into one block
void or_coarsen_block(void* hp, const int* kid4, double* out_avg, double* out_corner,
                      double* out_xedge, double* out_yedge) {
  Hier& h = *static_cast<Hier*>(hp);
  const Leaf* kids[2][2];
  for (int q = 0; q < 4; ++q) kids[q >> 1][q & 1] = &h.leaves[kid4[q]];
  Leaf C;
  h.alloc(C);
  coarsen_into(h, kids, C);
  double* outs[4] = {out_avg, out_corner, out_xedge, out_yedge};
  for (int k = 0; k < 4; ++k) std::memcpy(outs[k], C.blk[k].data(), C.blk[k].size() * sizeof(double));
}

}  // extern "C"

// ===========================================================================
// Learned regrid tagger: CPU reference (not part of the paper's method).
//
// Network: three 3x3 convolutions with zero "same" padding on 16x16 inputs
// (13 -> 32 -> 32 -> 32 channels), each followed by ReLU; global average
// pooling; a linear head 32 -> 3 (logits for coarsen / keep / refine);
// softmax cross-entropy averaged over the batch.  Layout NCHW, parameters
// W_l[co][ci][ky][kx], b_l[co], Wh[3][32], bh[3], packed in that order.
// With `bf16` set, every convolution operand (layer input and weight) is
// rounded first to FP32 and then to BF16 (round to nearest even), as the GPU
// path does; all arithmetic is FP64.
// ===========================================================================
namespace {

constexpr int kImg = 16, kPix = kImg * kImg, kWidth = 32, kClasses = 3;

double round_bf16(double v) {
  float f = float(v);
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return f;  // inf / nan unchanged
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  u &= 0xffff0000u;
  std::memcpy(&f, &u, 4);
  return f;
}

struct CnnShape {
  int cin[3], cout[3];
  size_t off_w[3], off_b[3], off_wh, off_bh, total;
};

CnnShape cnn_shape(int nin) {
  CnnShape s;
  size_t o = 0;
  for (int l = 0; l < 3; ++l) {
    s.cin[l] = l == 0 ? nin : kWidth;
    s.cout[l] = kWidth;
    s.off_w[l] = o;
    o += size_t(s.cout[l]) * s.cin[l] * 9;
    s.off_b[l] = o;
    o += s.cout[l];
  }
  s.off_wh = o;
  o += size_t(kClasses) * kWidth;
  s.off_bh = o;
  o += kClasses;
  s.total = o;
  return s;
}

// out[co][p] = b[co] + sum_{ci,ky,kx} in[ci][p + (ky-1, kx-1)] w[co][ci][ky][kx]
void conv3(const double* in, int cin, const double* w, const double* b, int cout, bool bf16, double* out) {
  for (int co = 0; co < cout; ++co)
    for (int y = 0; y < kImg; ++y)
      for (int x = 0; x < kImg; ++x) {
        double s = b[co];
        for (int ci = 0; ci < cin; ++ci)
          for (int ky = 0; ky < 3; ++ky)
            for (int kx = 0; kx < 3; ++kx) {
              const int yy = y + ky - 1, xx = x + kx - 1;
              if (yy < 0 || yy >= kImg || xx < 0 || xx >= kImg) continue;
              double a = in[size_t(ci) * kPix + yy * kImg + xx];
              double ww = w[((size_t(co) * cin + ci) * 3 + ky) * 3 + kx];
              if (bf16) {
                a = round_bf16(a);
                ww = round_bf16(ww);
              }
              s += a * ww;
            }
        out[size_t(co) * kPix + y * kImg + x] = s;
      }
}

struct CnnTape {
  std::vector<double> a[4];  // a[0] input, a[l] post-ReLU output of layer l
  std::vector<double> z[3];  // pre-activations
  double pooled[kWidth], logits[kClasses], prob[kClasses];
};

// Global mean pooling of a3, the linear head and the softmax.
void head_forward(const CnnShape& S, const double* P, CnnTape& T) {
  for (int c = 0; c < kWidth; ++c) {
    double s = 0.0;
    for (int p = 0; p < kPix; ++p) s += T.a[3][size_t(c) * kPix + p];
    T.pooled[c] = s / kPix;
  }
  double mx = -1e300;
  for (int k = 0; k < kClasses; ++k) {
    double s = P[S.off_bh + k];
    for (int c = 0; c < kWidth; ++c) s += P[S.off_wh + size_t(k) * kWidth + c] * T.pooled[c];
    T.logits[k] = s;
    mx = std::max(mx, s);
  }
  double den = 0.0;
  for (int k = 0; k < kClasses; ++k) den += std::exp(T.logits[k] - mx);
  for (int k = 0; k < kClasses; ++k) T.prob[k] = std::exp(T.logits[k] - mx) / den;
}

void cnn_forward_one(const CnnShape& S, const double* P, const double* x, bool bf16, CnnTape& T) {
  T.a[0].assign(x, x + size_t(S.cin[0]) * kPix);
  for (int l = 0; l < 3; ++l) {
    T.z[l].assign(size_t(S.cout[l]) * kPix, 0.0);
    conv3(T.a[l].data(), S.cin[l], P + S.off_w[l], P + S.off_b[l], S.cout[l], bf16, T.z[l].data());
    T.a[l + 1].resize(T.z[l].size());
    for (size_t i = 0; i < T.z[l].size(); ++i) T.a[l + 1][i] = T.z[l][i] > 0.0 ? T.z[l][i] : 0.0;
  }
  head_forward(S, P, T);
}

// d(loss_b / B) through the softmax, the head and the pooling: adds the head
// parameters' gradient to grad, writes the gradient with respect to a3 of
// this sample ([32][16][16]) to da, returns loss_b.
double head_backward(const CnnShape& S, const double* P, const CnnTape& T, int label, int B, double* grad,
                     double* da) {
  // d loss_b / d logits = prob - onehot, scaled by 1/B
  double dlog[kClasses];
  for (int k = 0; k < kClasses; ++k) dlog[k] = (T.prob[k] - (k == label ? 1.0 : 0.0)) / B;
  double dpool[kWidth] = {};
  for (int k = 0; k < kClasses; ++k) {
    grad[S.off_bh + k] += dlog[k];
    for (int c = 0; c < kWidth; ++c) {
      grad[S.off_wh + size_t(k) * kWidth + c] += dlog[k] * T.pooled[c];
      dpool[c] += dlog[k] * P[S.off_wh + size_t(k) * kWidth + c];
    }
  }
  // through the pooling: every pixel of channel c gets dpool[c]/256
  for (int c = 0; c < kWidth; ++c)
    for (int p = 0; p < kPix; ++p) da[size_t(c) * kPix + p] = dpool[c] / kPix;
  return -std::log(T.prob[label]);
}

// Adjoint of conv3 for one sample: with dz the gradient of the loss with
// respect to the output (pre-activation) [cout][16][16], adds
// d/dw = sum_p dz * in (shifted) to gW, d/db = sum_p dz to gb, and
// d/din = sum dz * w to din.  With bf16 the products use BF16-rounded
// operands (dz, in, w), as the forward products do.
void conv3_backward(const double* in, int cin, const double* W, const double* dz, int cout, bool bf16, double* gW,
                    double* gb, double* din) {
  for (int co = 0; co < cout; ++co)
    for (int y = 0; y < kImg; ++y)
      for (int x = 0; x < kImg; ++x) {
        gb[co] += dz[size_t(co) * kPix + y * kImg + x];
        double g = dz[size_t(co) * kPix + y * kImg + x];
        if (bf16) g = round_bf16(g);
        for (int ci = 0; ci < cin; ++ci)
          for (int ky = 0; ky < 3; ++ky)
            for (int kx = 0; kx < 3; ++kx) {
              const int yy = y + ky - 1, xx = x + kx - 1;
              if (yy < 0 || yy >= kImg || xx < 0 || xx >= kImg) continue;
              double a = in[size_t(ci) * kPix + yy * kImg + xx];
              double w = W[((size_t(co) * cin + ci) * 3 + ky) * 3 + kx];
              if (bf16) {
                a = round_bf16(a);
                w = round_bf16(w);
              }
              gW[((size_t(co) * cin + ci) * 3 + ky) * 3 + kx] += g * a;
              din[size_t(ci) * kPix + yy * kImg + xx] += g * w;
            }
      }
}

}  // namespace

extern "C" {

int or_cnn_num_params(int nin) { return int(cnn_shape(nin).total); }

// x: [B][nin][16][16]; logits: [B][3]; returns the mean cross-entropy when
// labels (0 coarsen, 1 keep, 2 refine) are given, else 0.
double or_cnn_forward(int nin, const double* params, const double* x, int B, const int* labels, int bf16,
                      double* logits) {
  const CnnShape S = cnn_shape(nin);
  double loss = 0.0;
  for (int b = 0; b < B; ++b) {
    CnnTape T;
    cnn_forward_one(S, params, x + size_t(b) * nin * kPix, bf16 != 0, T);
    for (int k = 0; k < kClasses; ++k) logits[size_t(b) * kClasses + k] = T.logits[k];
    if (labels) loss -= std::log(T.prob[labels[b]]);
  }
  return labels ? loss / B : 0.0;
}

// Gradient of the mean cross-entropy with respect to all parameters
// (backpropagation through the network above).  Also returns the layer
// activations of sample 0 if acts != NULL: [z1, a1, z2, a2, z3, a3] each
// [32][16][16].
double or_cnn_grad(int nin, const double* params, const double* x, int B, const int* labels, int bf16,
                   double* grad, double* acts) {
  const CnnShape S = cnn_shape(nin);
  std::fill(grad, grad + S.total, 0.0);
  double loss = 0.0;
  const bool rb = bf16 != 0;
  for (int b = 0; b < B; ++b) {
    CnnTape T;
    cnn_forward_one(S, params, x + size_t(b) * nin * kPix, rb, T);
    if (acts && b == 0)
      for (int l = 0; l < 3; ++l) {
        std::copy(T.z[l].begin(), T.z[l].end(), acts + size_t(2 * l) * kWidth * kPix);
        std::copy(T.a[l + 1].begin(), T.a[l + 1].end(), acts + size_t(2 * l + 1) * kWidth * kPix);
      }
    std::vector<double> da(size_t(kWidth) * kPix);
    loss += head_backward(S, params, T, labels[b], B, grad, da.data());
    for (int l = 2; l >= 0; --l) {
      // through the ReLU
      std::vector<double> dz(da.size());
      for (size_t i = 0; i < da.size(); ++i) dz[i] = T.z[l][i] > 0.0 ? da[i] : 0.0;
      std::vector<double> dain(size_t(S.cin[l]) * kPix, 0.0);
      conv3_backward(T.a[l].data(), S.cin[l], params + S.off_w[l], dz.data(), S.cout[l], rb, grad + S.off_w[l],
                     grad + S.off_b[l], dain.data());
      da.swap(dain);
    }
  }
  return loss / B;
}

// Backward of one 3x3 convolution layer (the adjoint of conv3) for a batch:
// in [B][cin][16][16] is the layer's input, dz [B][32][16][16] the gradient
// of the loss with respect to its pre-activation.  Adds to gW [32][cin][3][3]
// and gb [32], writes din [B][cin][16][16] (gradient with respect to the
// input).  With bf16 the operands of the products are rounded as in the
// forward pass; the bias gradient sums dz itself.
void or_cnn_conv_backward(const double* in, int B, int cin, const double* w, const double* dz, int bf16, double* gW,
                          double* gb, double* din) {
  for (int s = 0; s < B; ++s) {
    std::fill(din + size_t(s) * cin * kPix, din + size_t(s + 1) * cin * kPix, 0.0);
    conv3_backward(in + size_t(s) * cin * kPix, cin, w, dz + size_t(s) * kWidth * kPix, kWidth, bf16 != 0, gW, gb,
                   din + size_t(s) * cin * kPix);
  }
}

// Pooling, linear head and softmax cross-entropy of a batch from the last
// layer's post-activation a3 [B][32][16][16]: logits [B][3], the mean loss
// (returned), its gradient with respect to Wh [3][32] and bh [3] (added), and
// with respect to a3 (written, [B][32][16][16]).
double or_cnn_head(int nin, const double* params, const double* a3, int B, const int* labels, double* logits,
                   double* gWh, double* gbh, double* da3) {
  const CnnShape S = cnn_shape(nin);
  std::vector<double> g(S.total, 0.0);
  double loss = 0.0;
  for (int b = 0; b < B; ++b) {
    CnnTape T;
    T.a[3].assign(a3 + size_t(b) * kWidth * kPix, a3 + size_t(b + 1) * kWidth * kPix);
    head_forward(S, params, T);
    for (int k = 0; k < kClasses; ++k) logits[size_t(b) * kClasses + k] = T.logits[k];
    loss += head_backward(S, params, T, labels[b], B, g.data(), da3 + size_t(b) * kWidth * kPix);
  }
  for (int k = 0; k < kClasses; ++k) {
    gbh[k] += g[S.off_bh + k];
    for (int c = 0; c < kWidth; ++c) gWh[size_t(k) * kWidth + c] += g[S.off_wh + size_t(k) * kWidth + c];
  }
  return loss / B;
}

double or_round_bf16(double v) { return round_bf16(v); }

// One 3x3 convolution with bias (no activation): in [B][cin][16][16],
// w [32][cin][3][3], b [32], out [B][32][16][16].
void or_cnn_conv(const double* in, int B, int cin, const double* w, const double* b, int bf16, double* out) {
  for (int s = 0; s < B; ++s)
    conv3(in + size_t(s) * cin * kPix, cin, w, b, kWidth, bf16 != 0, out + size_t(s) * kWidth * kPix);
}

}  // extern "C"
