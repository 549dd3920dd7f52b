// af_internal.h -- definitions shared by the library's host code and its
// HIP kernels (never by anything outside libaf.so).
#pragma once

#include <cstdint>
#include <cstddef>

namespace af {

constexpr int kGhost = 2;          // two ghost layers (Sec. 3.2)
constexpr int kMaxLevels = 13;     // levels 0..12
constexpr int kThreads = 256;      // block size of every kernel (4 wave64)

// Raw DOFs of one cell in the order used by every stencil table:
// 0 avg, 1 corner(i,j), 2 corner(i+1,j), 3 corner(i,j+1), 4 corner(i+1,j+1),
// 5 xedge(i,j), 6 xedge(i+1,j), 7 yedge(i,j), 8 yedge(i,j+1).
constexpr int kCellDofs = 9;

// Node kinds (also the af.h AF_CORNER/AF_XEDGE/AF_YEDGE indices minus one).
enum NodeKind { NK_CORNER = 0, NK_XEDGE = 1, NK_YEDGE = 2 };

// Neighbourhood of raw DOFs entering the acoustic evolution of a node owned
// by cell (i,j): the union of the raw DOFs of the cells adjacent to the node
// (four for a corner, two for an edge midpoint).  Each entry is
// (state kind 0..3, di, dj) relative to (i,j).
struct NbEntry {
  int8_t kind, di, dj;
};
constexpr int kNbCorner = 25;
constexpr int kNbEdge = 15;

// corner (i,j): cells (i-1..i, j-1..j)
constexpr NbEntry kNbCornerTab[kNbCorner] = {
    {0, -1, -1}, {0, 0, -1}, {0, -1, 0}, {0, 0, 0},
    {1, -1, -1}, {1, 0, -1}, {1, 1, -1}, {1, -1, 0}, {1, 0, 0}, {1, 1, 0},
    {1, -1, 1}, {1, 0, 1}, {1, 1, 1},
    {2, -1, -1}, {2, 0, -1}, {2, 1, -1}, {2, -1, 0}, {2, 0, 0}, {2, 1, 0},
    {3, -1, -1}, {3, 0, -1}, {3, -1, 0}, {3, 0, 0}, {3, -1, 1}, {3, 0, 1}};
// xedge (i,j): cells (i-1,j), (i,j)
constexpr NbEntry kNbXedgeTab[kNbEdge] = {
    {0, -1, 0}, {0, 0, 0},
    {1, -1, 0}, {1, 0, 0}, {1, 1, 0}, {1, -1, 1}, {1, 0, 1}, {1, 1, 1},
    {2, -1, 0}, {2, 0, 0}, {2, 1, 0},
    {3, -1, 0}, {3, 0, 0}, {3, -1, 1}, {3, 0, 1}};
// yedge (i,j): cells (i,j-1), (i,j)
constexpr NbEntry kNbYedgeTab[kNbEdge] = {
    {0, 0, -1}, {0, 0, 0},
    {1, 0, -1}, {1, 1, -1}, {1, 0, 0}, {1, 1, 0}, {1, 0, 1}, {1, 1, 1},
    {2, 0, -1}, {2, 1, -1}, {2, 0, 0}, {2, 1, 0},
    {3, 0, -1}, {3, 0, 0}, {3, 0, 1}};

// Mirror orbits of the acoustic neighbourhoods.  The reflections x -> -x and
// y -> -y about a node map its neighbourhood onto itself, each DOF onto a DOF
// of the same kind, and commute with the sector means of eq. sphe-mean (the
// sectors of a node are mirror images).  So on an orbit of the reflections
// the K weights are equal, the Dx weights are odd in x and even in y, and
// the Dy weights even in x and odd in y (Dx vanishes where the offset from
// the node is 0 in x, Dy where it is 0 in y).  A node value is then a sum
// over orbits of K times the orbit sum plus Dx (Dy) times the orbit's
// x-odd (y-odd) sum.
//
// Offsets from the node in half-cell units of DOF (kind, di, dj) of the
// neighbourhood of node kind nk owned by cell (0,0).
constexpr void nb_offset(int nk, int kind, int di, int dj, int* X, int* Y) {
  // positions in half cells: x_{i-1/2} -> 2i, x_i -> 2i + 1
  const int px = 2 * di + ((kind == 0 || kind == 3) ? 1 : 0);
  const int py = 2 * dj + ((kind == 0 || kind == 2) ? 1 : 0);
  const int nx = nk == 2 ? 1 : 0, ny = nk == 1 ? 1 : 0;  // the node itself
  *X = px - nx;
  *Y = py - ny;
}

struct OrbitMember {
  int8_t kind, di, dj;
};
struct NbOrbit {
  int8_t n;           // 1, 2 or 4 members
  int8_t hasx, hasy;  // the members' offsets from the node are nonzero in x / in y
  // members in the order (+x, +y), (-x, +y), (+x, -y), (-x, -y), those with
  // a zero offset component left out
  OrbitMember m[4];
};
constexpr int kMaxOrbits = 9;
struct OrbitTable {
  int n;
  NbOrbit o[kMaxOrbits];
};

constexpr NbEntry nb_entry(int nk, int e) {
  return nk == 0 ? kNbCornerTab[e] : (nk == 1 ? kNbXedgeTab[e] : kNbYedgeTab[e]);
}
constexpr int nb_size(int nk) { return nk == 0 ? kNbCorner : kNbEdge; }
constexpr int iabs_c(int v) { return v < 0 ? -v : v; }

constexpr OrbitTable make_orbits(int nk) {
  OrbitTable T{};
  bool used[kNbCorner] = {};
  for (int e = 0; e < nb_size(nk); ++e) {
    if (used[e]) continue;
    const NbEntry E = nb_entry(nk, e);
    int X = 0, Y = 0;
    nb_offset(nk, E.kind, E.di, E.dj, &X, &Y);
    const int ax = iabs_c(X), ay = iabs_c(Y);
    NbOrbit O{};
    O.hasx = ax != 0;
    O.hasy = ay != 0;
    for (int sy = 1; sy >= -1; sy -= 2) {
      if (ay == 0 && sy < 0) continue;
      for (int sx = 1; sx >= -1; sx -= 2) {
        if (ax == 0 && sx < 0) continue;
        for (int f = 0; f < nb_size(nk); ++f) {
          const NbEntry G = nb_entry(nk, f);
          int gx = 0, gy = 0;
          nb_offset(nk, G.kind, G.di, G.dj, &gx, &gy);
          if (G.kind == E.kind && gx == sx * ax && gy == sy * ay) {
            used[f] = true;
            O.m[O.n++] = OrbitMember{G.kind, G.di, G.dj};
          }
        }
      }
    }
    T.o[T.n++] = O;
  }
  return T;
}
constexpr OrbitTable kOrbitTab[3] = {make_orbits(0), make_orbits(1), make_orbits(2)};
constexpr bool orbits_complete() {
  for (int nk = 0; nk < 3; ++nk) {
    int cnt = 0;
    for (int o = 0; o < kOrbitTab[nk].n; ++o) {
      const NbOrbit& O = kOrbitTab[nk].o[o];
      if (O.n != (O.hasx ? 2 : 1) * (O.hasy ? 2 : 1)) return false;
      cnt += O.n;
    }
    if (cnt != nb_size(nk)) return false;
  }
  return kOrbitTab[0].n == 9 && kOrbitTab[1].n == 6 && kOrbitTab[2].n == 6;
}
static_assert(orbits_complete(), "every neighbourhood entry lies in exactly one mirror orbit");

// Acoustic stencils in orbit form: [node kind][orbit][c][K, Dx, Dy] with
// c = 0 the value at t + dt and c = 1 the Simpson time sum without its term
// at t, 4 q(t + dt/2) + q(t + dt).
template <typename T>
struct AcOrbitWeights {
  T w[3][kMaxOrbits][2][3];
};

// Stencil weights of one level's step (same on every level under 2:1
// subcycling, since dt/dx is fixed).  Index [kind][tau] with tau 0 = dt/2,
// 1 = dt.
template <typename T>
struct AdvWeights {
  T w[3][2][kCellDofs];     // weights of the source cell's raw DOFs
  int32_t off[3][2][2];     // source cell offset (di, dj) from the owner cell
  // Upwind pattern only (sources (-1,-1), (-1,0), (0,-1) for corner, x-edge,
  // y-edge at both times): the new average of cell (0,0) as one linear
  // combination of the 25 old DOFs of the source cells (-1..0) x (-1..0):
  // index kUpA + (dj+1)*2 + (di+1) averages (di, dj in -1..0), kUpC +
  // (dj+1)*3 + (di+1) corners (di, dj in -1..1), kUpX + (dj+1)*3 + (di+1)
  // x-edges (di in -1..1, dj in -1..0), kUpY + (dj+1)*2 + (di+1) y-edges
  // (di in -1..0, dj in -1..1).
  T up_avg[25];
};
constexpr int kUpA = 0, kUpC = 4, kUpX = 13, kUpY = 19;

// Acoustics: p = K.p - Dx.u - Dy.v ; u = K.u - Dx.p ; v = K.v - Dy.p
// (eq. ERFormula: K is M_R + R d/dR M_R, Dx and Dy are R M_R of the x- and
// y-derivative), each a vector over the node's neighbourhood.
template <typename T>
struct AcWeights {
  T corner[2][3][kNbCorner];  // [tau][K,Dx,Dy][entry]
  T xedge[2][3][kNbEdge];
  T yedge[2][3][kNbEdge];
};

// Both forms of one step's acoustic stencils: the dense tables (level
// advance) and the orbit form (patch steps).
template <typename T>
struct AcAllWeights {
  AcWeights<T> dense;
  AcOrbitWeights<T> orbit;
};

// Device tables of a hierarchy.
struct HierDev {
  const int32_t* lut;        // per-level dense patch lookup: leaf id or -1
  const int32_t* plevel;     // [nleaves]
  const int32_t* pix;
  const int32_t* piy;
  int32_t lut_off[kMaxLevels];
  int32_t npx0, npy0, lmax, nleaves;
};

// Coarse-fine face for the conservative fix, grouped by coarse cell.
struct CFFace {
  int32_t coarse, side, k;   // coarse leaf, side (W,E,S,N), cell index along the side
  int32_t fine, fk;          // fine leaf facing it, index of the first of two fine faces
};

// Solid-body rotation (Sec. 4.2) for one step: the node positions of a patch
// and the rotation that traces a node back over tau = dt/2 (index 0) and dt
// (index 1).
template <typename T>
struct RotParams {
  T cs[2], sn[2];     // cos, sin of omega tau
  T x0, y0, dx, dy;   // domain origin, cell size of the level
  T omega, xc, yc;    // a = -omega (y - yc), b = omega (x - xc)
};

// Swirl flow (Sec. 4.3) for one step starting at time t: the velocity is the
// centred difference of Psi = sin^2(pi x) sin^2(pi y) cos(pi s) / pi over one
// cell; cos(pi s) is supplied for every time the step needs.
template <typename T>
struct SwirlParams {
  T x0, y0, dx, dy;  // domain origin, cell size of the level
  T kx, ky;          // sin(pi dx) / (pi dx), sin(pi dy) / (pi dy)
  T tau[2];          // dt/2, dt: the two traces back to t
  T cos_rk[2][3];    // cos(pi s) at the Runge-Kutta times t+tau, t+tau/2, t of each trace
  T cos_fx[3];       // cos(pi s) at t, t+dt/2, t+dt (Simpson times of the fluxes)
};

// Burgers (Sec. 2.2): tau / dx and tau / dy for tau = dt/2 and dt.
template <typename T>
struct BurgersParams {
  T tdx[2], tdy[2];
};

// Ghost-fill plan: one op per fill-set DOF of every leaf, holding the source
// that the fill rules resolve to for a given lower bound on source levels.
//   x: source leaf, or -1 for "keep the target's own value"
//   y: fill_info(op, source kind, source level, position, phase)
//   z, w: source (i, j) -- the element, fine cell or coarse cell
enum FillOpKind { FO_COPY = 0, FO_MEAN4 = 1, FO_EVAL = 2, FO_QAVG = 3 };
constexpr int kFillPoints = 25;  // EVAL positions (xi, eta) in {-1, -1/2, 0, 1/2, 1}^2: cx + 5 cy
constexpr int kFillQuarters = 4; // QAVG quarter qx + 2 qy, at positions kFillPoints + ...
__host__ __device__ constexpr int32_t fill_info(int op, int skind, int slevel, int pos, int phase) {
  return op | (skind << 2) | (slevel << 4) | (pos << 8) | (phase << 16);
}

// Weights of a cell's raw DOFs (kCellDofs order) for the reconstruction at
// the 25 EVAL positions and for the averages over its 4 quarters.
struct FillWeights {
  double w[kFillPoints + kFillQuarters][kCellDofs];
};

// Regrid transfer descriptor for one new leaf.
struct Transfer {
  int32_t mode;       // 0 copy, 1 refine from parent, 2 coarsen from children
  int32_t src[4];     // old leaf ids (copy/refine: src[0]; coarsen: child (qy*2+qx))
  int32_t qx, qy;     // refine: quadrant of the parent
};

}  // namespace af
