// af_kernels.hip -- gfx950 kernels of the Active Flux patch-step library.
//
// Every kernel uses 256-thread blocks (four 64-wide wavefronts).  State
// arrays are structure-of-arrays: four DOF kinds, each [ncomp][npatch]
// [m+5][pitch] (see include/af.h).
#include <hip/hip_runtime.h>

#include <mutex>
#include <type_traits>

#include "af_internal.h"
#include "af_launch.h"

namespace af {

// ---------------------------------------------------------------------------
// Patch step (Sec. 2): reconstruction + point-value evolution + Simpson flux
// + conservative update, for a tile of TY rows of one patch.
//
// A block stages rows [jlo-1, jhi+1] x cols [ilo-1, ihi+1] of all four DOF
// kinds in LDS, evaluates the owned point values of the "extended" cells
// [ilo,ihi] x [jlo,jhi] at t+dt/2 and t+dt, keeps their Simpson time sums
// (n + 4 (n+1/2) + (n+1)) in LDS, and updates the averages of cells
// [ilo,ihi) x [jlo,jhi) from the face fluxes.  Face fluxes are formed by one
// helper from the same LDS operands on both sides of a face, so neighbouring
// cells (and neighbouring patches) see bitwise-identical fluxes.
// ---------------------------------------------------------------------------

template <typename T>
struct StepArgs {
  const T* in[4];
  T* out[4];
  const int32_t* leaf_xy;  // [npatch][2] patch (ix, iy); rotation only
  int32_t npatch, pitch, first, region;
  T dtdx, dtdy;            // dt/dx, dt/dy
  T a, b, c;               // physics
  double len_dt_x;         // dy * dt (x-faces)
  double len_dt_y;         // dx * dt (y-faces)
  double* reg;             // [npatch][4][M][ncomp] or null
  const uint8_t* side_mask;
  // > 0: the patches first .. first + gnx * gny - 1 are a complete periodic
  // level in row-major order, and cells outside a patch are read from its
  // neighbours' interiors (no ghost fill needed); 0: from its ghost layers
  int32_t gnx, gny;
};

// Row-major walk e = start, start + stride, ... over an nx-wide grid without
// a division per element: (x, y) advance by (stride mod nx, stride div nx)
// with a carry.
struct Walk2 {
  int x, y, dx, dy, nx;
  __device__ __forceinline__ Walk2(int start, int stride, int nx_) : nx(nx_) {
    y = start / nx;
    x = start - y * nx;
    dy = stride / nx;
    dx = stride - dy * nx;
  }
  __device__ __forceinline__ void next() {
    x += dx;
    y += dy;
    if (x >= nx) {
      x -= nx;
      ++y;
    }
  }
};

// Block gather of NPL planes of an NR x NC image into LDS [plane][row][col]:
// position (r, x) of plane p is read from plane(p) + pos(r, x).  A thread's
// positions are the same in every plane, so their source offsets are
// computed once; all loads are issued before the first store.
template <typename T, int NT, int NPL, int NR, int NC, typename Plane, typename Pos>
__device__ __forceinline__ void gather_planes(T* lds, Plane plane, Pos pos) {
  constexpr int PE = NR * NC;
  constexpr int PER = (PE + NT - 1) / NT;
  size_t off[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = int(threadIdx.x) + u * NT;
    const int r = e / NC, x = e - r * NC;
    off[u] = e < PE ? pos(r, x) : 0;
  }
  T v[NPL][PER];
#pragma unroll
  for (int p = 0; p < NPL; ++p) {
    const T* const b = plane(p);
#pragma unroll
    for (int u = 0; u < PER; ++u)
      if (u + 1 < PER || PE % NT == 0 || int(threadIdx.x) + u * NT < PE) v[p][u] = b[off[u]];
  }
#pragma unroll
  for (int p = 0; p < NPL; ++p)
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = int(threadIdx.x) + u * NT;
      if (u + 1 < PER || PE % NT == 0 || e < PE) lds[p * PE + e] = v[p][u];
    }
}

// Workgroups are handed to the 8 XCDs round-robin (workgroup b to XCD b % 8),
// each XCD with its own L2.  Block b takes work item xcd_patch(b, n), so
// that each XCD runs one contiguous run of items: with n = 8 q + r, XCD x
// gets the q + (x < r) items from x q + min(x, r) on.  Those are the tiles of
// one patch and bands of neighbouring patches (leaves are sorted by level
// and row), whose reads of each other's cells then meet in one L2.  The map
// is a bijection of [0, n) for every n.
__device__ __forceinline__ int xcd_patch(int b, int n) {
  constexpr int kXcd = 8;
  const int x = b % kXcd, q = n / kXcd, r = n - q * kXcd;
  return x * q + min(x, r) + b / kXcd;
}

// LDS of a patch step: the staged DOFs, then the nodes' time sums.
// kLdsAlias: the update reads only the averages and the sums, so the sums
// overwrite the staged node values once every node is evaluated; the block
// then holds 4 NCOMP NR NC values, not 7 NCOMP NR NC, and more blocks fit on
// a CU.  The first of a fused pair of substeps uses it too: its new node
// values wait in registers until the update is done and then replace the
// sums.  kLdsSwirl: separate sums, and the swirl's values at t+dt (tsum2);
// its update also reads the nodes at t.
enum StepLdsKind { kLdsAlias, kLdsSwirl };

template <typename T, int NCOMP, int NR, int NC, int KIND>
struct StepLds;

template <typename T, int NCOMP, int NR, int NC>
struct StepLds<T, NCOMP, NR, NC, kLdsAlias> {
  using TS = T[3][NCOMP][NR - 2][NC];
  static constexpr bool kSeparate = false;
  T in[4][NCOMP][NR][NC];
  __device__ __forceinline__ TS& tsum() { return *reinterpret_cast<TS*>(&in[1][0][0][0]); }
  __device__ __forceinline__ TS& tsum2() { return tsum(); }  // unused without the swirl
};

template <typename T, int NCOMP, int NR, int NC>
struct StepLds<T, NCOMP, NR, NC, kLdsSwirl> {
  using TS = T[3][NCOMP][NR - 2][NC];
  static constexpr bool kSeparate = true;
  T in[4][NCOMP][NR][NC];
  TS ts, ts2;
  __device__ __forceinline__ TS& tsum() { return ts; }
  __device__ __forceinline__ TS& tsum2() { return ts2; }
};

// Simpson space-time sum of one face from the time sums of its three nodes
// (eq. Simpson-2d without the 1/36 and the flux function).
template <typename T>
__device__ __forceinline__ T face_sum(T lo, T mid, T hi) {
  return (lo + T(4) * mid) + hi;
}

template <typename T, int NR, int NC>
__device__ __forceinline__ T adv_eval(const T (&s)[4][1][NR][NC], int r, int c, const T* w) {
  // raw-DOF order of af_internal.h: avg, corners ll, rl, lu, ru, xedges l, r, yedges b, t
  T v = w[0] * s[0][0][r][c];
  v += w[1] * s[1][0][r][c];
  v += w[2] * s[1][0][r][c + 1];
  v += w[3] * s[1][0][r + 1][c];
  v += w[4] * s[1][0][r + 1][c + 1];
  v += w[5] * s[2][0][r][c];
  v += w[6] * s[2][0][r][c + 1];
  v += w[7] * s[3][0][r][c];
  v += w[8] * s[3][0][r + 1][c];
  return v;
}

// Both time levels of a node kind evaluated from one source cell (the usual
// case): one pass over the 9 raw DOFs feeds both dot products.
template <typename T, int NR, int NC>
__device__ __forceinline__ void adv_eval2(const T (&s)[4][1][NR][NC], int r, int c, const T* w0, const T* w1,
                                          T* h, T* f) {
  const T d[9] = {s[0][0][r][c],     s[1][0][r][c],     s[1][0][r][c + 1], s[1][0][r + 1][c], s[1][0][r + 1][c + 1],
                  s[2][0][r][c],     s[2][0][r][c + 1], s[3][0][r][c],     s[3][0][r + 1][c]};
  T a = w0[0] * d[0], b = w1[0] * d[0];
#pragma unroll
  for (int k = 1; k < 9; ++k) {
    a += w0[k] * d[k];
    b += w1[k] * d[k];
  }
  *h = a;
  *f = b;
}

// Acoustic node evaluation (eq. ERFormula with the sector weights collapsed
// on the host): the neighbourhood walked row by row.  Each table is four
// rectangles of source offsets, one per DOF kind, listed row by row (checked
// below), so entry e follows from (kind, row, column).  Fully unrolled, the
// three node kinds keep 330 weights live, more than the scalar registers
// hold, and the compiler parks them in vector lanes and reads each back
// before its use.  Here the rows are a loop that is not unrolled: the
// weights of a row are uniform loads issued in the iteration that uses them.
struct NbRect {
  int di0, di1, dj0, dj1;
};
constexpr NbRect kNbRects[3][4] = {
    {{-1, 0, -1, 0}, {-1, 1, -1, 1}, {-1, 1, -1, 0}, {-1, 0, -1, 1}},  // corner
    {{-1, 0, 0, 0}, {-1, 1, 0, 1}, {-1, 1, 0, 0}, {-1, 0, 0, 1}},      // x-edge
    {{0, 0, -1, 0}, {0, 1, -1, 1}, {0, 1, -1, 0}, {0, 0, -1, 1}}};     // y-edge

template <int NB>
constexpr bool rects_match(int nk, const NbEntry (&tab)[NB]) {
  int e = 0;
  for (int kind = 0; kind < 4; ++kind) {
    const NbRect R = kNbRects[nk][kind];
    for (int dj = R.dj0; dj <= R.dj1; ++dj)
      for (int di = R.di0; di <= R.di1; ++di, ++e)
        if (e >= NB || tab[e].kind != kind || tab[e].di != di || tab[e].dj != dj) return false;
  }
  return e == NB;
}
static_assert(rects_match(0, kNbCornerTab) && rects_match(1, kNbXedgeTab) && rects_match(2, kNbYedgeTab),
              "neighbourhood tables are four row-major rectangles");

template <typename T, int NR, int NC, int NK, int NB>
__device__ __forceinline__ void ac_eval_rows(const T (&s)[4][3][NR][NC], int r, int c, const T (&w)[2][3][NB],
                                             T out[2][3]) {
  T kp[2] = {T(0), T(0)}, ku[2] = {T(0), T(0)}, kv[2] = {T(0), T(0)};
  T dxu[2] = {T(0), T(0)}, dyv[2] = {T(0), T(0)}, dxp[2] = {T(0), T(0)}, dyp[2] = {T(0), T(0)};
  int ebase = 0;
#pragma unroll
  for (int kind = 0; kind < 4; ++kind) {
    const NbRect R = kNbRects[NK][kind];
    const int ndi = R.di1 - R.di0 + 1;
#pragma unroll 1
    for (int dj = R.dj0; dj <= R.dj1; ++dj) {
      const int e0 = ebase + (dj - R.dj0) * ndi;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        if (q >= ndi) break;
        const int di = R.di0 + q;
        const T p = s[kind][0][r + dj][c + di], u = s[kind][1][r + dj][c + di], v = s[kind][2][r + dj][c + di];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const T wk = w[t][0][e0 + q], wx = w[t][1][e0 + q], wy = w[t][2][e0 + q];
          kp[t] += wk * p;
          ku[t] += wk * u;
          kv[t] += wk * v;
          dxu[t] += wx * u;
          dyv[t] += wy * v;
          dxp[t] += wx * p;
          dyp[t] += wy * p;
        }
      }
    }
    ebase += ndi * (R.dj1 - R.dj0 + 1);
  }
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    out[t][0] = kp[t] - dxu[t] - dyv[t];
    out[t][1] = ku[t] - dxp[t];
    out[t][2] = kv[t] - dyp[t];
  }
}

// Acoustic node evaluation in mirror-orbit form (af_internal.h): each node
// kind sums its neighbourhood orbit by orbit, reading an orbit's members
// from LDS just before use.  For an orbit of four members (+x,+y), (-x,+y),
// (+x,-y), (-x,-y) the sum, the x-odd sum and the y-odd sum take 7 additions
// from the pair sums and differences; K multiplies the sum of every
// component, Dx the x-odd sums of u (into p) and p (into u), Dy the y-odd
// sums of v (into p) and p (into v).
// v1: the node's value at t + dt; vs: 4 q(t + dt/2) + q(t + dt).
// Orbit o of node kind NK added to acc: the orbit sum S and odd parts Dx,
// Dy of the neighbourhood values, times the orbit's weights.
template <typename T, int NK, int NR, int NC>
__device__ __forceinline__ void ac_orbit(const T (&s)[4][3][NR][NC], int r, int c,
                                         const T (&w)[kMaxOrbits][2][3], int o, T (&acc)[2][3]) {
  const NbOrbit& O = kOrbitTab[NK].o[o];
  T S[3], Dx[3] = {T(0), T(0), T(0)}, Dy[3] = {T(0), T(0), T(0)};
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const T m0 = s[O.m[0].kind][q][r + O.m[0].dj][c + O.m[0].di];
    if (O.n == 1) {
      S[q] = m0;
    } else if (O.n == 2) {
      const T m1 = s[O.m[1].kind][q][r + O.m[1].dj][c + O.m[1].di];
      S[q] = m0 + m1;
      if (O.hasx && q != 2) Dx[q] = m0 - m1;
      if (O.hasy && q != 1) Dy[q] = m0 - m1;
    } else {
      const T m1 = s[O.m[1].kind][q][r + O.m[1].dj][c + O.m[1].di];
      const T m2 = s[O.m[2].kind][q][r + O.m[2].dj][c + O.m[2].di];
      const T m3 = s[O.m[3].kind][q][r + O.m[3].dj][c + O.m[3].di];
      const T hi = m0 + m1, lo = m2 + m3;
      S[q] = hi + lo;
      if (q != 1) Dy[q] = hi - lo;
      if (q != 2) Dx[q] = (m0 - m1) + (m2 - m3);
    }
  }
#pragma unroll
  for (int cc = 0; cc < 2; ++cc) {
    const T wk = w[o][cc][0], wx = w[o][cc][1], wy = w[o][cc][2];
    acc[cc][0] += wk * S[0];
    acc[cc][1] += wk * S[1];
    acc[cc][2] += wk * S[2];
    if (O.hasx) {
      acc[cc][0] -= wx * Dx[1];
      acc[cc][1] -= wx * Dx[0];
    }
    if (O.hasy) {
      acc[cc][0] -= wy * Dy[2];
      acc[cc][2] -= wy * Dy[0];
    }
  }
}

// Orbits [O0, O1) of node kind NK added to acc.
template <typename T, int NK, int NR, int NC, int O0, int O1>
__device__ __forceinline__ void ac_orbit_range(const T (&s)[4][3][NR][NC], int r, int c,
                                               const T (&w)[kMaxOrbits][2][3], T (&acc)[2][3]) {
#pragma unroll
  for (int o = O0; o < O1; ++o) ac_orbit<T, NK, NR, NC>(s, r, c, w, o, acc);
}

template <typename T, int NK, int NR, int NC>
__device__ __forceinline__ void ac_node(const T (&s)[4][3][NR][NC], int r, int c,
                                        const T (&w)[kMaxOrbits][2][3], T v1[3], T vs[3]) {
  T acc[2][3] = {{T(0), T(0), T(0)}, {T(0), T(0), T(0)}};
#pragma unroll
  for (int o = 0; o < kOrbitTab[NK].n; ++o) ac_orbit<T, NK, NR, NC>(s, r, c, w, o, acc);
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    v1[q] = acc[0][q];
    vs[q] = acc[1][q];
  }
}

template <typename T, int EQ>
struct WSel;
template <typename T>
struct WSel<T, 0> { using type = AdvWeights<T>; };
template <typename T>
struct WSel<T, 1> { using type = AcOrbitWeights<T>; };
template <typename T>
struct WSel<T, 2> { using type = RotParams<T>; };
template <typename T>
struct WSel<T, 3> { using type = SwirlParams<T>; };
template <typename T>
struct WSel<T, 4> { using type = BurgersParams<T>; };

constexpr double kPiD = 3.14159265358979323846264338327950288;

// Swirl velocity (Sec. 4.3, eq. swirlODE): centred differences over one
// cell of the level of Psi = sin^2(pi x) sin^2(pi y) cos(pi t) / pi.  With
// sin^2 A - sin^2 B = sin(A + B) sin(A - B) the differences are products,
//   a = -cos(pi t) ky sin^2(pi x) sin(2 pi y),
//   b =  cos(pi t) kx sin(2 pi x) sin^2(pi y),   k = sin(pi h) / (pi h),
// the same numbers without the cancellation of the difference of two close
// values (which costs FP32 about log10(1/h) digits) and with two sincospi
// calls instead of eight sines.
__device__ __forceinline__ void sincos_pi(float v, float* s, float* c) { sincospif(v, s, c); }
__device__ __forceinline__ void sincos_pi(double v, double* s, double* c) { sincospi(v, s, c); }

template <typename T>
__device__ __forceinline__ void swirl_vel(const SwirlParams<T>& W, T x, T y, T c, T* a, T* b) {
  T sx, cx, sy, cy;
  sincos_pi(x, &sx, &cx);
  sincos_pi(y, &sy, &cy);
  *a = -c * W.ky * (sx * sx) * (T(2) * sy * cy);
  *b = c * W.kx * (T(2) * sx * cx) * (sy * sy);
}

// Cell of a foot at coordinate s (cell units: cell k spans [k-1/2, k+1/2])
// and the reference coordinate in it; a foot on a face goes to the cell
// between it and the node (disp = node - foot), as for constant advection.
template <typename T>
__device__ __forceinline__ int foot_cell(T s, T disp) {
  return int(disp < T(0) ? ceil(s + T(0.5)) - T(1) : floor(s + T(0.5)));
}

// Reconstruction (Sec. 2, eq. poly) of the staged cell at LDS (r, c),
// evaluated at reference point (xi, eta): tensor Lagrange interpolant of the
// 9 nodal values, centre value from "average = Simpson sum".
template <typename T, int NR, int NC>
__device__ __forceinline__ T rot_eval(const T (&s)[4][1][NR][NC], int r, int c, T xi, T eta) {
  const T lx[3] = {T(0.5) * xi * (xi - T(1)), T(1) - xi * xi, T(0.5) * xi * (xi + T(1))};
  const T ly[3] = {T(0.5) * eta * (eta - T(1)), T(1) - eta * eta, T(0.5) * eta * (eta + T(1))};
  T q[3][3];  // [x node][y node]
  q[0][0] = s[1][0][r][c];
  q[2][0] = s[1][0][r][c + 1];
  q[0][2] = s[1][0][r + 1][c];
  q[2][2] = s[1][0][r + 1][c + 1];
  q[0][1] = s[2][0][r][c];
  q[2][1] = s[2][0][r][c + 1];
  q[1][0] = s[3][0][r][c];
  q[1][2] = s[3][0][r + 1][c];
  q[1][1] = (T(36) * s[0][0][r][c] - (q[0][0] + q[2][0] + q[0][2] + q[2][2]) -
             T(4) * (q[0][1] + q[2][1] + q[1][0] + q[1][2])) / T(16);
  T v = T(0);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) v += q[a][b] * lx[a] * ly[b];
  return v;
}

// The compute part of a patch step on a staged block (shared by the one-level
// kernel k_patch_step and the multi-level kernel k_amr_step): point values of
// the extended cells [ilo, ihi] x [jlo, jhi] at t + dt/2 and t + dt, their
// Simpson time sums in LDS, then fluxes and the conservative update of cells
// [ilo, ihi) x [jlo, jhi), flux registers of the patch's boundary faces.
template <typename T>
struct StepIO {
  T* out[4];               // the output state (patch planes at patch, component stride npatch planes)
  int32_t npatch, pitch, patch, region;
  T dtdx, dtdy, a, b, c;
  double len_dt_x, len_dt_y;  // dy * dt, dx * dt of the patch's level
  double* reg;             // FP64 registers [npatch][4][M][NCOMP]; null: nothing recorded
  uint32_t smask;          // sides whose faces are recorded
};

// TO_LDS: the first substep of a fused pair (no HBM output): new node values
// and averages replace the staged ones in L.in.  The time sums are aliased
// onto the staged nodes, so the node values go in after the update, which
// reads the sums from where they will be stored.  rofs: staged row of cell
// row j is j - jlo + 1 + rofs (the pair's second substep reads the first's
// rows).
template <typename T, int EQ, int M, int TY, bool TO_LDS = false, typename L_t>
__device__ __forceinline__ void step_compute(L_t& L, const StepIO<T>& A, const typename WSel<T, EQ>::type& W,
                                             int jlo, int jhi, T px0, T py0, int rofs = 0) {
  static_assert(!TO_LDS || ((EQ == 0 || EQ == 1) && !L_t::kSeparate),
                "a fused pair needs a constant-coefficient equation and the aliased LDS layout");
  constexpr int NCOMP = EQ == 1 ? 3 : 1;
  constexpr int NR = TY + 3;
  constexpr int NC = M + 5;
  const int patch = A.patch;
  const int region = A.region;
  const int ilo = -region, ihi = M + region;
  const int span = ihi - ilo;
  const int nrow = jhi - jlo;
  const size_t plane = size_t(M + 5) * A.pitch;
  const int coff = ilo + 2;  // staged column of cell i is i + 2 = ii + coff

  // ---- point values of the extended cells [ilo, ihi] x [jlo, jhi]
  const int EC = span + 1, ER = nrow + 1;
  const bool last_tile = (jhi == ihi);
  bool shared_src = true;  // uniform: both time levels read the same source cell
  if constexpr (EQ == 0) {
#pragma unroll
    for (int kind = 0; kind < 3; ++kind)
      shared_src = shared_src && W.off[kind][0][0] == W.off[kind][1][0] && W.off[kind][0][1] == W.off[kind][1][1];
  }
  // the extended cells of a thread: at most MAXIT (region <= 1, nrow <= TY);
  // their time sums wait in registers until every node is evaluated.  The
  // acoustic node pass walks rows of the LDS pitch NC (the columns past EC
  // idle): the 64 lanes of a wave then read 64 consecutive LDS values at
  // every stencil point, free of bank conflicts (rows of EC on a pitch of NC
  // wrap onto the banks of the wave's first lanes).  The time sums are
  // stored on the same pitch.
  constexpr bool kWide = EQ == 1;
  const int WN = kWide ? NC : EC;
  constexpr int MAXIT = ((kWide ? M + 5 : M + 3) * (TY + 1) + kThreads - 1) / kThreads;
  T tsv[MAXIT][3][NCOMP];
  T nv[TO_LDS ? MAXIT : 1][3][NCOMP];  // TO_LDS: the new node values, stored after the barrier
  // a new node value: to HBM (if `keep`, the rows and columns this tile
  // owns), or held for LDS
  auto emit = [&](int it, int kind, int q, bool keep, size_t o, T v) {
    if constexpr (TO_LDS) {
      nv[it][kind][q] = v;
    } else {
      if (keep) A.out[kind + 1][o] = v;
    }
  };
  Walk2 w(threadIdx.x, kThreads, WN);
#pragma unroll
  for (int it = 0; it < MAXIT; ++it, w.next()) {
    if (w.y >= ER) break;
    if (kWide && w.x >= EC) continue;
    const int ii = w.x, jj = w.y;
    const int i = ilo + ii, j = jlo + jj;
    const int r = jj + 1 + rofs, c = ii + coff;  // staged position of cell (i,j)
    const bool wrow = (jj < nrow) || last_tile;
    const bool has_x = jj < nrow;      // xedge (i,j) belongs to rows [jlo, jhi)
    const bool has_y = ii < span;      // yedge (i,j) belongs to cols [ilo, ihi)
    const size_t obase = size_t(j + kGhost) * A.pitch + (i + kGhost);
    if constexpr (EQ == 0) {
#pragma unroll
      for (int kind = 0; kind < 3; ++kind) {
        if (kind == NK_XEDGE && !has_x) continue;
        if (kind == NK_YEDGE && !has_y) continue;
        T h, f;
        if (shared_src) {
          adv_eval2<T, NR, NC>(L.in, r + W.off[kind][0][1], c + W.off[kind][0][0], W.w[kind][0], W.w[kind][1], &h, &f);
        } else {
          h = adv_eval<T, NR, NC>(L.in, r + W.off[kind][0][1], c + W.off[kind][0][0], W.w[kind][0]);
          f = adv_eval<T, NR, NC>(L.in, r + W.off[kind][1][1], c + W.off[kind][1][0], W.w[kind][1]);
        }
        const T cur = L.in[kind + 1][0][r][c];
        tsv[it][kind][0] = (cur + T(4) * h) + f;
        emit(it, kind, 0, wrow, size_t(patch) * plane + obase, f);
      }
    } else if constexpr (EQ == 2 || EQ == 3) {
      // solid-body rotation (Sec. 4.2): the foot is the node turned back by
      // -omega tau about (xc, yc); swirl (Sec. 4.3): one classical Runge-Kutta
      // step back along the characteristic.  q^n there from its cell's
      // reconstruction.
#pragma unroll
      for (int kind = 0; kind < 3; ++kind) {
        if (kind == NK_XEDGE && !has_x) continue;
        if (kind == NK_YEDGE && !has_y) continue;
        const T X = kind == NK_YEDGE ? T(i) : T(i) - T(0.5);  // node in cell units
        const T Y = kind == NK_XEDGE ? T(j) : T(j) - T(0.5);
        const T x = px0 + (X + T(0.5)) * W.dx, y = py0 + (Y + T(0.5)) * W.dy;
        T val[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          T fx, fy;
          if constexpr (EQ == 2) {
            const T rx = x - W.xc, ry = y - W.yc;
            fx = W.xc + rx * W.cs[t] + ry * W.sn[t];
            fy = W.yc - rx * W.sn[t] + ry * W.cs[t];
          } else {
            const T h = -W.tau[t];
            T a1, b1, a2, b2, a3, b3, a4, b4;
            swirl_vel(W, x, y, W.cos_rk[t][0], &a1, &b1);
            swirl_vel(W, x + T(0.5) * h * a1, y + T(0.5) * h * b1, W.cos_rk[t][1], &a2, &b2);
            swirl_vel(W, x + T(0.5) * h * a2, y + T(0.5) * h * b2, W.cos_rk[t][1], &a3, &b3);
            swirl_vel(W, x + h * a3, y + h * b3, W.cos_rk[t][2], &a4, &b4);
            fx = x + h / T(6) * (a1 + T(2) * a2 + T(2) * a3 + a4);
            fy = y + h / T(6) * (b1 + T(2) * b2 + T(2) * b3 + b4);
          }
          const T sx = (fx - px0) / W.dx - T(0.5), sy = (fy - py0) / W.dy - T(0.5);
          // source cell, kept in the range a Courant number <= 1 allows
          // (the halo holds it): nodes on x-faces i-1..i, else i-1..i+1
          int ci = foot_cell(sx, x - fx), cj = foot_cell(sy, y - fy);
          ci = min(max(ci, i - 1), kind == NK_YEDGE ? i + 1 : i);
          cj = min(max(cj, j - 1), kind == NK_XEDGE ? j + 1 : j);
          val[t] = rot_eval<T, NR, NC>(L.in, r + (cj - j), c + (ci - i), T(2) * (sx - T(ci)), T(2) * (sy - T(cj)));
        }
        if constexpr (EQ == 2) {
          const T cur = L.in[kind + 1][0][r][c];
          tsv[it][kind][0] = (cur + T(4) * val[0]) + val[1];
        } else {
          tsv[it][kind][0] = val[0];
          L.tsum2()[kind][0][jj][ii] = val[1];
        }
        if (wrow) A.out[kind + 1][size_t(patch) * plane + obase] = val[1];
      }
    } else if constexpr (EQ == 4) {
      // Burgers (Sec. 2.2): the point value solves q = q^n(P - q tau (1, 1));
      // two fixed-point iterations from the mean of the averages around the
      // node.  The time sum holds the fluxes q^2/2 (Simpson in time).
      const auto& av = L.in[0][0];
#pragma unroll
      for (int kind = 0; kind < 3; ++kind) {
        if (kind == NK_XEDGE && !has_x) continue;
        if (kind == NK_YEDGE && !has_y) continue;
        T Q0;
        if (kind == NK_CORNER) {
          Q0 = T(0.25) * ((av[r][c - 1] + av[r][c]) + (av[r - 1][c - 1] + av[r - 1][c]));
        } else if (kind == NK_XEDGE) {
          Q0 = T(0.5) * (av[r][c - 1] + av[r][c]);
        } else {
          Q0 = T(0.5) * (av[r][c] + av[r - 1][c]);
        }
        const T X = kind == NK_YEDGE ? T(i) : T(i) - T(0.5);  // node in cell units
        const T Y = kind == NK_XEDGE ? T(j) : T(j) - T(0.5);
        T val[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          T Q = Q0;
#pragma unroll
          for (int it = 0; it < 2; ++it) {
            const T sx = X - Q * W.tdx[t], sy = Y - Q * W.tdy[t];
            // source cell, kept in the range a Courant number <= 1 allows
            int ci = foot_cell(sx, Q), cj = foot_cell(sy, Q);
            ci = min(max(ci, i - 1), kind == NK_YEDGE ? i + 1 : i);
            cj = min(max(cj, j - 1), kind == NK_XEDGE ? j + 1 : j);
            Q = rot_eval<T, NR, NC>(L.in, r + (cj - j), c + (ci - i), T(2) * (sx - T(ci)), T(2) * (sy - T(cj)));
          }
          val[t] = Q;
        }
        const T cur = L.in[kind + 1][0][r][c];
        tsv[it][kind][0] = (T(0.5) * cur * cur + T(2) * val[0] * val[0]) + T(0.5) * val[1] * val[1];
        if (wrow) A.out[kind + 1][size_t(patch) * plane + obase] = val[1];
      }
    }
  }
  if constexpr (EQ == 1) {
    // acoustics (eq. ERFormula): one node kind at a time over the thread's
    // cells, each node from its neighbourhood orbit by orbit.  The kind's
    // orbit weights (42 for a corner, 26 for an edge) fit in scalar
    // registers for the whole pass and the FP32 kernel needs about 90 VGPRs,
    // not 126 (5 waves per SIMD, not 4).  An FP64 weight takes two scalar
    // registers, so FP64 sums a node's orbits in two ranges, each with its
    // own weight loads: the kernel then fits 168 VGPRs (3 waves per SIMD,
    // not 2).
    auto kind_pass = [&](auto kc) {
      constexpr int K = decltype(kc)::value;
      Walk2 v(threadIdx.x, kThreads, WN);
#pragma unroll
      for (int it = 0; it < MAXIT; ++it, v.next()) {
        if (v.y >= ER) break;
        if (kWide && v.x >= EC) continue;
        const int ii = v.x, jj = v.y;
        if (K == NK_XEDGE && jj >= nrow) continue;  // x-edges of rows [jlo, jhi)
        if (K == NK_YEDGE && ii >= span) continue;  // y-edges of cols [ilo, ihi)
        const int r = jj + 1 + rofs, c = ii + coff;
        const size_t obase = size_t(jlo + jj + kGhost) * A.pitch + (ilo + ii + kGhost);
        const bool wst = K == NK_XEDGE || jj < nrow || last_tile;
        T v1[3], vs[3];
        if constexpr (sizeof(T) == 8) {
          constexpr int H = K == NK_CORNER ? 5 : 3;
          T acc[2][3] = {{T(0), T(0), T(0)}, {T(0), T(0), T(0)}};
          ac_orbit_range<T, K, NR, NC, 0, H>(L.in, r, c, W.w[K], acc);
          ac_orbit_range<T, K, NR, NC, H, kOrbitTab[K].n>(L.in, r, c, W.w[K], acc);
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            v1[q] = acc[0][q];
            vs[q] = acc[1][q];
          }
        } else {
          ac_node<T, K, NR, NC>(L.in, r, c, W.w[K], v1, vs);
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          tsv[it][K][q] = L.in[K + 1][q][r][c] + vs[q];
          emit(it, K, q, wst, (size_t(q) * A.npatch + patch) * plane + obase, v1[q]);
        }
      }
    };
    kind_pass(std::integral_constant<int, NK_CORNER>());
    kind_pass(std::integral_constant<int, NK_XEDGE>());
    kind_pass(std::integral_constant<int, NK_YEDGE>());
  }
  __syncthreads();
  auto& ts = L.tsum();
  {
    Walk2 v(threadIdx.x, kThreads, WN);
#pragma unroll
    for (int it = 0; it < MAXIT; ++it, v.next()) {
      if (v.y >= ER) break;
      if (kWide && v.x >= EC) continue;
      const int ii = v.x, jj = v.y;
#pragma unroll
      for (int q = 0; q < NCOMP; ++q) {
        ts[NK_CORNER][q][jj][ii] = tsv[it][NK_CORNER][q];
        if (jj < nrow) ts[NK_XEDGE][q][jj][ii] = tsv[it][NK_XEDGE][q];
        if (ii < span) ts[NK_YEDGE][q][jj][ii] = tsv[it][NK_YEDGE][q];
      }
    }
  }
  __syncthreads();

  // ---- fluxes and conservative update (eq. 2dfv) of cells [ilo,ihi) x [jlo,jhi)
  const uint32_t smask = A.reg ? A.smask : 0u;
  const T inv36 = T(1) / T(36);
  for (Walk2 w(threadIdx.x, kThreads, span); w.y < nrow; w.next()) {
    const int ii = w.x, jj = w.y;
    const int i = ilo + ii, j = jlo + jj;
    const size_t obase = size_t(j + kGhost) * A.pitch + (i + kGhost);
    T FL[NCOMP], FR[NCOMP], GB[NCOMP], GT[NCOMP];
#pragma unroll
    for (int q = 0; q < NCOMP; ++q) {
      FL[q] = face_sum(ts[NK_CORNER][q][jj][ii], ts[NK_XEDGE][q][jj][ii], ts[NK_CORNER][q][jj + 1][ii]);
      FR[q] = face_sum(ts[NK_CORNER][q][jj][ii + 1], ts[NK_XEDGE][q][jj][ii + 1],
                       ts[NK_CORNER][q][jj + 1][ii + 1]);
      GB[q] = face_sum(ts[NK_CORNER][q][jj][ii], ts[NK_YEDGE][q][jj][ii], ts[NK_CORNER][q][jj][ii + 1]);
      GT[q] = face_sum(ts[NK_CORNER][q][jj + 1][ii], ts[NK_YEDGE][q][jj + 1][ii],
                       ts[NK_CORNER][q][jj + 1][ii + 1]);
    }
    // physical fluxes of the Simpson sums: advection f = a q, g = b q;
    // acoustics f = c (u, p, 0), g = c (v, 0, p)  (Sec. 2.3)
    T fL[NCOMP], fR[NCOMP], gB[NCOMP], gT[NCOMP];
    if constexpr (EQ == 0) {
      fL[0] = A.a * FL[0] * inv36; fR[0] = A.a * FR[0] * inv36;
      gB[0] = A.b * GB[0] * inv36; gT[0] = A.b * GT[0] * inv36;
    } else if constexpr (EQ == 3) {
      // swirl (eq. swirlF, swirlG): the face-midpoint velocity at t, t+dt/2,
      // t+dt times the Simpson sum of the three nodes at that time
      const int rr = jj + 1 + rofs, cc = ii + coff;  // staged position of cell (i, j)
      const auto& Q0 = L.in;
      const auto& Qh = ts;
      const auto& Qf = L.tsum2();
      const T xl = px0 + T(i) * W.dx, xr = px0 + T(i + 1) * W.dx, xm = px0 + (T(i) + T(0.5)) * W.dx;
      const T yb = py0 + T(j) * W.dy, yt = py0 + T(j + 1) * W.dy, ym = py0 + (T(j) + T(0.5)) * W.dy;
      // the spatial factors of the face-midpoint velocities, then one
      // cos(pi s) per Simpson time
      T sxl, cxl, sxr, cxr, sxm, cxm, syb, cyb, syt, cyt, sym, cym;
      sincos_pi(xl, &sxl, &cxl);
      sincos_pi(xr, &sxr, &cxr);
      sincos_pi(xm, &sxm, &cxm);
      sincos_pi(yb, &syb, &cyb);
      sincos_pi(yt, &syt, &cyt);
      sincos_pi(ym, &sym, &cym);
      const T s2ym = T(2) * sym * cym, s2xm = T(2) * sxm * cxm;
      const T AL = -W.ky * (sxl * sxl) * s2ym, AR = -W.ky * (sxr * sxr) * s2ym;
      const T BB = W.kx * s2xm * (syb * syb), BT = W.kx * s2xm * (syt * syt);
      T aL[3], aR[3], bB[3], bT[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        aL[k] = W.cos_fx[k] * AL;
        aR[k] = W.cos_fx[k] * AR;
        bB[k] = W.cos_fx[k] * BB;
        bT[k] = W.cos_fx[k] * BT;
      }
      const T SL[3] = {face_sum(Q0[1][0][rr][cc], Q0[2][0][rr][cc], Q0[1][0][rr + 1][cc]),
                       face_sum(Qh[NK_CORNER][0][jj][ii], Qh[NK_XEDGE][0][jj][ii], Qh[NK_CORNER][0][jj + 1][ii]),
                       face_sum(Qf[NK_CORNER][0][jj][ii], Qf[NK_XEDGE][0][jj][ii], Qf[NK_CORNER][0][jj + 1][ii])};
      const T SR[3] = {face_sum(Q0[1][0][rr][cc + 1], Q0[2][0][rr][cc + 1], Q0[1][0][rr + 1][cc + 1]),
                       face_sum(Qh[NK_CORNER][0][jj][ii + 1], Qh[NK_XEDGE][0][jj][ii + 1], Qh[NK_CORNER][0][jj + 1][ii + 1]),
                       face_sum(Qf[NK_CORNER][0][jj][ii + 1], Qf[NK_XEDGE][0][jj][ii + 1], Qf[NK_CORNER][0][jj + 1][ii + 1])};
      const T SB[3] = {face_sum(Q0[1][0][rr][cc], Q0[3][0][rr][cc], Q0[1][0][rr][cc + 1]),
                       face_sum(Qh[NK_CORNER][0][jj][ii], Qh[NK_YEDGE][0][jj][ii], Qh[NK_CORNER][0][jj][ii + 1]),
                       face_sum(Qf[NK_CORNER][0][jj][ii], Qf[NK_YEDGE][0][jj][ii], Qf[NK_CORNER][0][jj][ii + 1])};
      const T ST[3] = {face_sum(Q0[1][0][rr + 1][cc], Q0[3][0][rr + 1][cc], Q0[1][0][rr + 1][cc + 1]),
                       face_sum(Qh[NK_CORNER][0][jj + 1][ii], Qh[NK_YEDGE][0][jj + 1][ii], Qh[NK_CORNER][0][jj + 1][ii + 1]),
                       face_sum(Qf[NK_CORNER][0][jj + 1][ii], Qf[NK_YEDGE][0][jj + 1][ii], Qf[NK_CORNER][0][jj + 1][ii + 1])};
      fL[0] = (aL[0] * SL[0] + T(4) * aL[1] * SL[1] + aL[2] * SL[2]) * inv36;
      fR[0] = (aR[0] * SR[0] + T(4) * aR[1] * SR[1] + aR[2] * SR[2]) * inv36;
      gB[0] = (bB[0] * SB[0] + T(4) * bB[1] * SB[1] + bB[2] * SB[2]) * inv36;
      gT[0] = (bT[0] * ST[0] + T(4) * bT[1] * ST[1] + bT[2] * ST[2]) * inv36;
    } else if constexpr (EQ == 4) {
      // Burgers: the time sums already hold f = g = q^2/2
      fL[0] = FL[0] * inv36; fR[0] = FR[0] * inv36;
      gB[0] = GB[0] * inv36; gT[0] = GT[0] * inv36;
    } else if constexpr (EQ == 2) {
      // rotation: f = a(node) q with a = -omega (y - yc) on x-faces (a depends
      // on y only) and g = b(node) q with b = omega (x - xc) on y-faces
      const T a0 = -W.omega * (py0 + T(j) * W.dy - W.yc);
      const T a1 = -W.omega * (py0 + (T(j) + T(0.5)) * W.dy - W.yc);
      const T a2 = -W.omega * (py0 + T(j + 1) * W.dy - W.yc);
      const T b0 = W.omega * (px0 + T(i) * W.dx - W.xc);
      const T b1 = W.omega * (px0 + (T(i) + T(0.5)) * W.dx - W.xc);
      const T b2 = W.omega * (px0 + T(i + 1) * W.dx - W.xc);
      fL[0] = (a0 * ts[NK_CORNER][0][jj][ii] + T(4) * a1 * ts[NK_XEDGE][0][jj][ii] + a2 * ts[NK_CORNER][0][jj + 1][ii]) * inv36;
      fR[0] = (a0 * ts[NK_CORNER][0][jj][ii + 1] + T(4) * a1 * ts[NK_XEDGE][0][jj][ii + 1] +
               a2 * ts[NK_CORNER][0][jj + 1][ii + 1]) * inv36;
      gB[0] = (b0 * ts[NK_CORNER][0][jj][ii] + T(4) * b1 * ts[NK_YEDGE][0][jj][ii] + b2 * ts[NK_CORNER][0][jj][ii + 1]) * inv36;
      gT[0] = (b0 * ts[NK_CORNER][0][jj + 1][ii] + T(4) * b1 * ts[NK_YEDGE][0][jj + 1][ii] +
               b2 * ts[NK_CORNER][0][jj + 1][ii + 1]) * inv36;
    } else {
      fL[0] = A.c * FL[1] * inv36; fL[1] = A.c * FL[0] * inv36; fL[2] = T(0);
      fR[0] = A.c * FR[1] * inv36; fR[1] = A.c * FR[0] * inv36; fR[2] = T(0);
      gB[0] = A.c * GB[2] * inv36; gB[1] = T(0); gB[2] = A.c * GB[0] * inv36;
      gT[0] = A.c * GT[2] * inv36; gT[1] = T(0); gT[2] = A.c * GT[0] * inv36;
    }
#pragma unroll
    for (int q = 0; q < NCOMP; ++q) {
      const T Q = L.in[0][q][jj + 1 + rofs][ii + coff];
      const T Qn = Q - A.dtdx * (fR[q] - fL[q]) - A.dtdy * (gT[q] - gB[q]);
      if constexpr (TO_LDS) {
        L.in[0][q][jj + 1 + rofs][ii + coff] = Qn;  // read only by this thread
      } else {
        A.out[0][(size_t(q) * A.npatch + patch) * plane + obase] = Qn;
      }
    }
    if (smask) {
      // boundary faces of the interior block -> FP64 registers (Sec. 3.2)
      double* R = A.reg + size_t(patch) * 4 * M * NCOMP;
      const bool interior = (i >= 0 && i < M && j >= 0 && j < M);
      if (interior) {
#pragma unroll
        for (int q = 0; q < NCOMP; ++q) {
          if (i == 0 && (smask & 1)) R[(0 * M + j) * NCOMP + q] += double(fL[q]) * A.len_dt_x;
          if (i == M - 1 && (smask & 2)) R[(1 * M + j) * NCOMP + q] += double(fR[q]) * A.len_dt_x;
          if (j == 0 && (smask & 4)) R[(2 * M + i) * NCOMP + q] += double(gB[q]) * A.len_dt_y;
          if (j == M - 1 && (smask & 8)) R[(3 * M + i) * NCOMP + q] += double(gT[q]) * A.len_dt_y;
        }
      }
    }
  }
  if constexpr (TO_LDS) {
    // the new node values of the extended cells, over the time sums
    __syncthreads();
    Walk2 v(threadIdx.x, kThreads, WN);
#pragma unroll
    for (int it = 0; it < MAXIT; ++it, v.next()) {
      if (v.y >= ER) break;
      if (kWide && v.x >= EC) continue;
      const int ii = v.x, jj = v.y;
      const int r = jj + 1 + rofs, c = ii + coff;
#pragma unroll
      for (int q = 0; q < NCOMP; ++q) {
        L.in[1][q][r][c] = nv[it][NK_CORNER][q];
        if (jj < nrow) L.in[2][q][r][c] = nv[it][NK_XEDGE][q];
        if (ii < span) L.in[3][q][r][c] = nv[it][NK_YEDGE][q];
      }
    }
  }
}


template <typename T, int EQ, int M, int TY, bool GN>
__global__ __launch_bounds__(kThreads) void k_patch_step(const StepArgs<T> A,
                                                         const typename WSel<T, EQ>::type W) {
  constexpr int NCOMP = EQ == 1 ? 3 : 1;
  constexpr int NR = TY + 3;
  constexpr int NC = M + 5;
  __shared__ StepLds<T, NCOMP, NR, NC, EQ == 3 ? kLdsSwirl : kLdsAlias> L;

  const int region = A.region;
  const int ilo = -region, ihi = M + region;
  const int span = ihi - ilo;
  const int tiles = (span + TY - 1) / TY;
  const int rows = (span + tiles - 1) / tiles;  // balanced tile height, at most TY
  const int w = xcd_patch(int(blockIdx.x), int(gridDim.x));
  const int pl = w / tiles;
  const int patch = A.first + pl;
  const int tile = w - pl * tiles;
  const int jlo = ilo + tile * rows;
  const int jhi = min(jlo + rows, ihi);
  if (jlo >= jhi) return;  // block-uniform; cannot happen for the compiled (m, TY) pairs
  const int nrow = jhi - jlo;
  const size_t plane = size_t(M + 5) * A.pitch;

  // ---- stage NR rows from j = jlo-1 (clamped to the array for a short last
  // tile) and all M+5 columns (staged column x holds i = x - 2), so the
  // image has a compile-time shape; rows [jlo-1, jhi+1] and columns
  // [ilo-1, ihi+1] are the ones read below
  if constexpr (GN) {  // cells outside the patch from its neighbours' interiors
    const int gpl = patch - A.first;
    const int pix = gpl % A.gnx, piy = gpl / A.gnx;
    // the source patch and offset of a position are the same for every
    // (kind, component) plane
    gather_planes<T, kThreads, 4 * NCOMP, NR, NC>(
        &L.in[0][0][0][0], [&](int p) { return A.in[p / NCOMP] + size_t(p % NCOMP) * A.npatch * plane; },
        [&](int rr, int x) {
          const int j = min(jlo - 1 + rr, M + 2), i = x - kGhost;
          const int oy = j < 0 ? -1 : (j >= M ? 1 : 0);
          const int ox = i < 0 ? -1 : (i >= M ? 1 : 0);
          int xx = pix + ox, yy = piy + oy;
          xx = xx < 0 ? xx + A.gnx : (xx >= A.gnx ? xx - A.gnx : xx);
          yy = yy < 0 ? yy + A.gny : (yy >= A.gny ? yy - A.gny : yy);
          const int src = A.first + yy * A.gnx + xx;
          return size_t(src) * plane + size_t(j - oy * M + kGhost) * A.pitch + (i - ox * M + kGhost);
        });
  } else {
    // the patch's own planes, (kind, component) in the image's order; rows
    // from jlo - 1, clamped to the array for a short last tile
    gather_planes<T, kThreads, 4 * NCOMP, NR, NC>(
        &L.in[0][0][0][0],
        [&](int p) { return A.in[p / NCOMP] + (size_t(p % NCOMP) * A.npatch + patch) * plane; },
        [&](int rr, int x) { return size_t(min(jlo - 1 + rr, M + 2) + kGhost) * A.pitch + x; });
  }
  __syncthreads();
  // rotation, swirl: lower-left corner of the patch's cell (0,0)
  T px0 = T(0), py0 = T(0);
  if constexpr (EQ == 2 || EQ == 3) {
    px0 = W.x0 + T(A.leaf_xy[2 * patch] * M) * W.dx;
    py0 = W.y0 + T(A.leaf_xy[2 * patch + 1] * M) * W.dy;
  }
  StepIO<T> io;
#pragma unroll
  for (int k = 0; k < 4; ++k) io.out[k] = A.out[k];
  io.npatch = A.npatch;
  io.pitch = A.pitch;
  io.patch = patch;
  io.region = region;
  io.dtdx = A.dtdx;
  io.dtdy = A.dtdy;
  io.a = A.a;
  io.b = A.b;
  io.c = A.c;
  io.len_dt_x = A.len_dt_x;
  io.len_dt_y = A.len_dt_y;
  io.reg = A.side_mask ? A.reg : nullptr;
  io.smask = (A.reg && A.side_mask) ? A.side_mask[patch] : 0u;
  step_compute<T, EQ, M, TY>(L, io, W, jlo, jhi, px0, py0);
}

// ---------------------------------------------------------------------------
// Level advance: K steps of every patch of a level whose eight neighbours
// are leaves of the same level, in one launch (temporal blocking).
//
// A block owns one patch.  It gathers the patch and a K-cell halo from the
// interiors of the 3x3 neighbourhood (each DOF from the patch owning its
// cell, Sec. 2 ownership: exactly the values a same-level ghost fill copies),
// then takes K steps in LDS on shrinking regions (step s updates cells
// [-(K-1-s), m+K-1-s)), and finally writes the interior averages and the
// closed-square nodes.  Step s reads only data of step s-1 that lie inside
// its own block, so K fused steps equal K separate fill+step passes.
//
// k_level_advance below is the acoustic kernel (three components, sector
// means); advection has its own layout in k_level_advance_adv.
// ---------------------------------------------------------------------------

template <typename T>
struct AdvanceArgs {
  const T* in[4];
  T* out[4];
  int32_t npatch, pitch, first;
  int32_t nx, ny;  // patches per side of the level; leaf first + iy * nx + ix is patch (ix, iy)
  T dtdx, dtdy, a, b, c;
};

// Patch index of the periodic neighbour (ox, oy) in {-1, 0, 1}^2 of patch
// (ix, iy) on a complete level stored in row-major order.
template <typename T>
__device__ __forceinline__ int level_nbr(const AdvanceArgs<T>& A, int ix, int iy, int ox, int oy) {
  int xx = ix + ox, yy = iy + oy;
  xx = xx < 0 ? xx + A.nx : (xx >= A.nx ? xx - A.nx : xx);
  yy = yy < 0 ? yy + A.ny : (yy >= A.ny ? yy - A.ny : yy);
  return A.first + yy * A.nx + xx;
}

template <typename T, int M, int K, int NT>
__global__ __launch_bounds__(NT) void k_level_advance(const AdvanceArgs<T> A, const AcWeights<T> W) {
  constexpr int NCOMP = 3;
  constexpr int E = M + 2 * K + 1;     // node extent of the gathered block
  constexpr int EMAX = M + 2 * K - 1;  // extended cells per side in the first step
  constexpr int CPT = (EMAX * EMAX + NT - 1) / NT;  // extended cells per thread (first step)
  __shared__ T st[4][NCOMP][E][E];
  __shared__ T ts[3][NCOMP][E][E];

  const int pl = xcd_patch(int(blockIdx.x), int(gridDim.x));
  const int patch = A.first + pl;
  const int pix = pl % A.nx, piy = pl / A.nx;
  const size_t plane = size_t(M + 5) * A.pitch;

  // ---- gather: LDS position (r, c) holds local index (c - K, r - K)
  gather_planes<T, NT, 4 * NCOMP, E, E>(
      &st[0][0][0][0], [&](int p) { return A.in[p / NCOMP] + size_t(p % NCOMP) * A.npatch * plane; },
      [&](int rr, int x) {
        const int j = rr - K, i = x - K;
        const int oy = j < 0 ? -1 : (j >= M ? 1 : 0);
        const int ox = i < 0 ? -1 : (i >= M ? 1 : 0);
        const int src = level_nbr(A, pix, piy, ox, oy);
        const int li = i - ox * M, lj = j - oy * M;
        return size_t(src) * plane + size_t(lj + kGhost) * A.pitch + (li + kGhost);
      });
  __syncthreads();

  const T inv36 = T(1) / T(36);
#pragma unroll 1
  for (int s = 0; s < K; ++s) {
    const int lo = -(K - 1 - s), hi = M + (K - 1 - s);
    const int EC = hi - lo + 1;
    T fnew[CPT][3][NCOMP];
    // ---- node values of the extended cells [lo, hi]^2
    {
      Walk2 w(threadIdx.x, NT, EC);
#pragma unroll
      for (int u = 0; u < CPT; ++u, w.next()) {
        const int ii = w.x, jj = w.y;
        if (jj >= EC) break;
        const int r = lo + jj + K, c = lo + ii + K;  // LDS position of cell (i, j)
        const bool has_x = jj < EC - 1, has_y = ii < EC - 1;
        {
          T res[2][3];
          ac_eval_rows<T, E, E, 0, kNbCorner>(st, r, c, W.corner, res);
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            ts[NK_CORNER][q][r][c] = (st[1][q][r][c] + T(4) * res[0][q]) + res[1][q];
            fnew[u][NK_CORNER][q] = res[1][q];
          }
          if (has_x) {
            ac_eval_rows<T, E, E, 1, kNbEdge>(st, r, c, W.xedge, res);
#pragma unroll
            for (int q = 0; q < 3; ++q) {
              ts[NK_XEDGE][q][r][c] = (st[2][q][r][c] + T(4) * res[0][q]) + res[1][q];
              fnew[u][NK_XEDGE][q] = res[1][q];
            }
          }
          if (has_y) {
            ac_eval_rows<T, E, E, 2, kNbEdge>(st, r, c, W.yedge, res);
#pragma unroll
            for (int q = 0; q < 3; ++q) {
              ts[NK_YEDGE][q][r][c] = (st[3][q][r][c] + T(4) * res[0][q]) + res[1][q];
              fnew[u][NK_YEDGE][q] = res[1][q];
            }
          }
        }
      }
    }
    __syncthreads();
    // ---- commit the new point values, then update the averages of [lo, hi)^2
    {
      Walk2 w(threadIdx.x, NT, EC);
#pragma unroll
      for (int u = 0; u < CPT; ++u, w.next()) {
        const int ii = w.x, jj = w.y;
        if (jj >= EC) break;
        const int r = lo + jj + K, c = lo + ii + K;
        const bool has_x = jj < EC - 1, has_y = ii < EC - 1;
#pragma unroll
        for (int q = 0; q < NCOMP; ++q) {
          st[1][q][r][c] = fnew[u][NK_CORNER][q];
          if (has_x) st[2][q][r][c] = fnew[u][NK_XEDGE][q];
          if (has_y) st[3][q][r][c] = fnew[u][NK_YEDGE][q];
        }
        if (!has_x || !has_y) continue;  // cells with i or j == hi are not updated
        T FL[NCOMP], FR[NCOMP], GB[NCOMP], GT[NCOMP];
#pragma unroll
        for (int q = 0; q < NCOMP; ++q) {
          FL[q] = face_sum(ts[NK_CORNER][q][r][c], ts[NK_XEDGE][q][r][c], ts[NK_CORNER][q][r + 1][c]);
          FR[q] = face_sum(ts[NK_CORNER][q][r][c + 1], ts[NK_XEDGE][q][r][c + 1], ts[NK_CORNER][q][r + 1][c + 1]);
          GB[q] = face_sum(ts[NK_CORNER][q][r][c], ts[NK_YEDGE][q][r][c], ts[NK_CORNER][q][r][c + 1]);
          GT[q] = face_sum(ts[NK_CORNER][q][r + 1][c], ts[NK_YEDGE][q][r + 1][c], ts[NK_CORNER][q][r + 1][c + 1]);
        }
        T fL[NCOMP], fR[NCOMP], gB[NCOMP], gT[NCOMP];
        fL[0] = A.c * FL[1] * inv36; fL[1] = A.c * FL[0] * inv36; fL[2] = T(0);
        fR[0] = A.c * FR[1] * inv36; fR[1] = A.c * FR[0] * inv36; fR[2] = T(0);
        gB[0] = A.c * GB[2] * inv36; gB[1] = T(0); gB[2] = A.c * GB[0] * inv36;
        gT[0] = A.c * GT[2] * inv36; gT[1] = T(0); gT[2] = A.c * GT[0] * inv36;
#pragma unroll
        for (int q = 0; q < NCOMP; ++q)
          st[0][q][r][c] = st[0][q][r][c] - A.dtdx * (fR[q] - fL[q]) - A.dtdy * (gT[q] - gB[q]);
      }
    }
    __syncthreads();
  }

  // ---- write the interior averages and the closed-square nodes
  constexpr int NN = (M + 1) * (M + 1);
  for (int e = threadIdx.x; e < NCOMP * NN; e += NT) {
    const int q = e / NN, f = e - q * NN;
    const int i = f % (M + 1), j = f / (M + 1);
    const int r = j + K, c = i + K;
    const size_t g = (size_t(q) * A.npatch + patch) * plane + size_t(j + kGhost) * A.pitch + (i + kGhost);
    A.out[1][g] = st[1][q][r][c];
    if (j < M) A.out[2][g] = st[2][q][r][c];
    if (i < M) A.out[3][g] = st[3][q][r][c];
    if (i < M && j < M) A.out[0][g] = st[0][q][r][c];
  }
}

// ---------------------------------------------------------------------------
// Level advance for advection (Sec. 2, eq. evolution by characteristics):
// the same K-step scheme as k_level_advance with a layout built for LDS
// latency rather than capacity.
//
//  * Point values are double-buffered (pt[s & 1] old, pt[~s & 1] new), so
//    the node pass writes new values straight to LDS and the update pass only
//    touches time sums and averages; nothing is held in registers across the
//    barrier.
//  * A cell's node pass loads all 27 source DOFs of its three node kinds
//    before any arithmetic, so the pass pays the LDS latency once.
//  * Every array has R spare rows.  Strips of R rows that run past a region
//    store into positions that no later read touches: regions shrink by one
//    cell per side and step, and a window reaches one cell past its region,
//    so anything outside the current extended region, and the top-row
//    x-edges and right-column y-edges in it, is never read again.  The
//    strided passes store without selects.
//  * The K steps are unrolled: region sizes and the buffer parity are
//    compile-time, so every LDS address is a per-task base plus an
//    immediate.
//  * SS: both time levels of a node kind share one source cell (always true
//    when the transverse Courant number is at most 1/2), one load feeds both
//    dot products.
//  * The upwind pattern (a, b > 0 with both directional Courant numbers
//    below 1/2: sources corner (i-1, j-1), x-edge (i-1, j), y-edge (i, j-1))
//    runs in k_level_advance_up instead, one pass per step.
//  * A wave whose 64 cells of a slot all lie outside the region skips it.
// ---------------------------------------------------------------------------

// Source-cell offset (d = 0: di, d = 1: dj) of the upwind pattern for node kind k.
__host__ __device__ constexpr int up_off(int k, int d) { return k == NK_CORNER ? -1 : (k == NK_XEDGE ? d - 1 : -d); }

// Rows per strip: a thread takes R vertically adjacent cells of one column,
// with R the smallest value that lets one pass of NT threads cover the first
// (largest) region.
template <int M, int K, int NT>
struct StripRows {
  static constexpr int EC0 = M + 2 * K - 1;
  static constexpr int S = NT / EC0 > 0 ? NT / EC0 : 1;
  static constexpr int R0 = (EC0 + S - 1) / S;
  static constexpr int value = R0 > 6 ? 6 : R0;
};

template <typename T, int M, int K, int R>
struct AdvLds {
  static constexpr int E = M + 2 * K + 1;
  static constexpr int ER = E + R;  // rows of every array: E, then R spare rows for strips past a region
  T av[ER][E];        // averages; av, pt[0][0..2] are the gather targets (stride ER * E)
  T pt[2][3][ER][E];  // point values, [buffer][kind]
  T ts[3][ER][E];     // Simpson time sums n + 4 (n+1/2) + (n+1)
};

template <typename T, int M, int K, int NT, bool SS>
__global__ __launch_bounds__(NT) void k_level_advance_adv(const AdvanceArgs<T> A, const AdvWeights<T> W) {
  constexpr int R = StripRows<M, K, NT>::value;
  using L = AdvLds<T, M, K, R>;
  constexpr int E = L::E;
  constexpr int EE = E * E;
  constexpr int AS = L::ER * E;  // stride between arrays
  __shared__ L S;

  const int pl = xcd_patch(int(blockIdx.x), int(gridDim.x));
  const int patch = A.first + pl;
  const int pix = pl % A.nx, piy = pl / A.nx;
  const size_t plane = size_t(M + 5) * A.pitch;

  // ---- gather: LDS position (r, c) holds local index (c - K, r - K);
  // kind 0 goes to av, kinds 1..3 to pt[0][0..2] (stride AS after av).  A
  // thread takes positions tid, tid + NT, ...; one source offset serves the
  // four kinds, and every load is issued before the first store
  T* const g0 = &S.av[0][0];
  {
    constexpr int NP = (EE + NT - 1) / NT;
    T v[NP][4];
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      const int e = int(threadIdx.x) + u * NT;
      if (u + 1 < NP || EE % NT == 0 || e < EE) {
        const int rr = e / E, x = e - rr * E;
        const int j = rr - K, i = x - K;
        const int oy = j < 0 ? -1 : (j >= M ? 1 : 0);
        const int ox = i < 0 ? -1 : (i >= M ? 1 : 0);
        const int src = level_nbr(A, pix, piy, ox, oy);
        const size_t off = size_t(src) * plane + size_t(j - oy * M + kGhost) * A.pitch + (i - ox * M + kGhost);
#pragma unroll
        for (int kind = 0; kind < 4; ++kind) v[u][kind] = A.in[kind][off];
      }
    }
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      const int e = int(threadIdx.x) + u * NT;
      if (u + 1 < NP || EE % NT == 0 || e < EE) {
#pragma unroll
        for (int kind = 0; kind < 4; ++kind) g0[kind * AS + e] = v[u][kind];
      }
    }
  }
  __syncthreads();

  const T inv36 = T(1) / T(36);
  const T cx = A.dtdx * A.a * inv36, cy = A.dtdy * A.b * inv36;
#pragma unroll
  for (int s = 0; s < K; ++s) {
    T* const avp = &S.av[0][0];
    const T* const po = &S.pt[s & 1][0][0][0];
    T* const pn = &S.pt[(s + 1) & 1][0][0][0];
    T* const tsp = &S.ts[0][0][0];
    const int lo = -(K - 1 - s);
    const int EC = M + 2 * (K - 1 - s) + 1;  // extended cells per side
    const int base = (lo + K) * (E + 1);      // LDS index of the first extended cell
    const int nslot = (EC * EC + NT - 1) / NT;
    // ---- node values of the extended cells
    Walk2 w(threadIdx.x, NT, EC);
#pragma unroll 1
    for (int u = 0; u < nslot; ++u, w.next()) {
      if (u * NT + int(threadIdx.x & ~63u) >= EC * EC) break;  // wave-uniform
      const bool ok = w.y < EC;
      const int ii = ok ? w.x : 0, jj = ok ? w.y : 0;
      const int idx = base + jj * E + ii;
      const bool has_x = ok && jj < EC - 1, has_y = ok && ii < EC - 1;
      T d[3][9], d1[3][9];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
#pragma unroll
        for (int t = 0; t < (SS ? 1 : 2); ++t) {
          // source cell; the clamp only moves sources of nodes that are not
          // kept (top-row x-edge, right-column y-edge), so that their DOFs
          // (r + 1, c + 1) stay inside the array
          int si = idx + W.off[k][t][1] * E + W.off[k][t][0];
          si = min(si, EE - E - 2);
          T* dd = t ? d1[k] : d[k];
          dd[0] = avp[si];
          dd[1] = po[si];
          dd[2] = po[si + 1];
          dd[3] = po[si + E];
          dd[4] = po[si + E + 1];
          dd[5] = po[AS + si];
          dd[6] = po[AS + si + 1];
          dd[7] = po[2 * AS + si];
          dd[8] = po[2 * AS + si + E];
        }
      }
      T own[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) own[k] = po[k * AS + idx];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const T* dh = d[k];
        const T* df = SS ? d[k] : d1[k];
        T h = W.w[k][0][0] * dh[0], f = W.w[k][1][0] * df[0];
#pragma unroll
        for (int e = 1; e < 9; ++e) {
          h += W.w[k][0][e] * dh[e];
          f += W.w[k][1][e] * df[e];
        }
        const bool keep = k == NK_CORNER ? ok : (k == NK_XEDGE ? has_x : has_y);
        const int o = keep ? idx : 0;
        tsp[k * AS + o] = (own[k] + T(4) * h) + f;
        pn[k * AS + o] = f;
      }
    }
    __syncthreads();
    // ---- conservative update of cells [lo, hi)^2 (EC - 1 per side), in
    // strips of R rows; the y-face between two rows of a strip is summed once
    {
      const int NC = EC - 1;
      const int ns = (NC + R - 1) / R;
      const int ntask = NC * ns;
#pragma unroll 1
      for (int t0 = 0; t0 + int(threadIdx.x & ~63u) < ntask; t0 += NT) {  // wave-uniform
        const int t = t0 + int(threadIdx.x);
        const bool tok = t < ntask;
        const int q = tok ? t / NC : 0;
        const int ci = tok ? t - q * NC : 0;
        const int b0 = base + q * R * E + ci;
        T G[R + 1], FL[R], FR[R], Q[R];  // every load before the first store
#pragma unroll
        for (int u = 0; u <= R; ++u)
          G[u] = face_sum(tsp[b0 + u * E], tsp[2 * AS + b0 + u * E], tsp[b0 + u * E + 1]);
#pragma unroll
        for (int u = 0; u < R; ++u) {
          const int idx = b0 + u * E;
          FL[u] = face_sum(tsp[idx], tsp[AS + idx], tsp[idx + E]);
          FR[u] = face_sum(tsp[idx + 1], tsp[AS + idx + 1], tsp[idx + E + 1]);
          Q[u] = avp[idx];
        }
        if (tok) {  // rows past the region land in rows no later read touches
#pragma unroll
          for (int u = 0; u < R; ++u) avp[b0 + u * E] = (Q[u] - cx * (FR[u] - FL[u])) - cy * (G[u + 1] - G[u]);
        }
      }
    }
    __syncthreads();
  }

  // ---- write the interior averages and the closed-square nodes
  const T* const pf = &S.pt[K & 1][0][0][0];
  for (Walk2 w(threadIdx.x, NT, M + 1); w.y < M + 1; w.next()) {
    const int i = w.x, j = w.y;
    const int idx = (j + K) * E + (i + K);
    const size_t g = size_t(patch) * plane + size_t(j + kGhost) * A.pitch + (i + kGhost);
    A.out[1][g] = pf[idx];
    if (j < M) A.out[2][g] = pf[AS + idx];
    if (i < M) A.out[3][g] = pf[2 * AS + idx];
    if (i < M && j < M) A.out[0][g] = g0[idx];
  }
}

// ---------------------------------------------------------------------------
// Level advance for advection with the upwind source pattern in one pass per
// step.  With constant velocity each node value at t + dt/2 and t + dt is a
// fixed combination of its source cell's DOFs, so the update of eq. 2dfv
// over the Simpson sums (eq. Simpson-2d) of a cell's eight face nodes is one
// fixed combination of the 25 old DOFs of its source cells (-1..0)^2,
// composed on the host (AdvWeights::up_avg).  A cell's new average and its
// three new node values come from the same window of old DOFs.  Averages
// and point values are double-buffered: a step reads one buffer, writes the
// other, and needs one barrier and no time sums.  A thread takes a strip of
// R vertically adjacent cells of one column; strips that run past the
// region store into spare rows that no later window reads.
//
// Region.  The dependence grows by one cell per step on the upwind side only.
// The write-back stores averages at i, j < M, corners at i, j <= M, x-edge
// values at i <= M, j < M and y-edge values at i < M, j <= M.  In x, each of
// these reads only averages and y-edge values at i < M and corners and
// x-edge values at i <= M (the sources are cells i - 1 and i of the new
// average, and cell i - 1 or i of a node at index i); y is the same with the
// edge kinds swapped.  So step s computes local cells s + 1 - K .. M in each
// direction, a side of M + K - s, and the gather reads local -K .. M.  The
// column and row just past a region are read but never written: the
// averages and edge values at index M that come from them are not among
// the ones above, and nothing needed reads them.
//
// LDS layouts.  Step s reads layout s and writes layout s + 1; the layouts
// alternate between the two buffers.  Layout s puts local cell (s - K, s - K)
// at position 0 and has row pitch pitch(s): the gather fills layout 0, the
// write-back reads layout K.  Most shapes instead store the last step's
// region, the closed square, to the output directly (UpGeom::DIRECT).  Step
// s gives each strip width(s) consecutive tasks (its region width, rounded
// up to a multiple of gcd(R, B), where B is the number of elements that
// cover the 32 LDS banks once) and pitch(s) is
// the smallest pitch with R * pitch(s) = width(s) modulo B.  The address of
// task t is then t plus a constant modulo B, across strip boundaries, so the
// window loads of any 32 (FP32) or 16 (FP64) consecutive lanes fall in
// distinct banks.
// ---------------------------------------------------------------------------
template <typename T, int M, int K, int R>
struct UpPlan {
  static constexpr int E0 = M + K + 1;  // side of the gathered block
  static constexpr int B = 128 / int(sizeof(T));
  static constexpr int gcd(int a, int b) { return b == 0 ? a : gcd(b, a % b); }
  static constexpr int ec(int s) { return M + K - s; }  // region side of step s
  static constexpr int width(int s) {
    int w = ec(s);
    while (w % gcd(R, B) != 0) ++w;
    return w;
  }
  static constexpr int pitch(int s) {
    // layout s must hold the columns step s - 1 writes (ec(s - 1)); layout 0
    // the gathered block, layout K the closed square of M + 1 nodes
    int p = s == 0 ? E0 : (s == K ? M + 1 : ec(s - 1));
    if (s == K) return p;
    for (int i = 0; i < B && (R * p - width(s)) % B != 0; ++i) ++p;
    return p;
  }
  static constexpr bool valid() {
    for (int s = 0; s < K; ++s)
      if ((R * pitch(s) - width(s)) % B != 0) return false;
    return true;
  }
  static constexpr int max_pitch() {
    int m = 0;
    for (int s = 0; s <= K; ++s) m = pitch(s) > m ? pitch(s) : m;
    return m;
  }
  static constexpr int strips(int s) { return (ec(s) + R - 1) / R; }
  // words of one array of layout s that anything touches: the gather (s = 0)
  // or step s - 1 writes, step s reads (its last strip's window reaches row
  // strips * R + 1 and, from idle columns, column width + 1), the write-back
  // reads the closed square (s = K)
  static constexpr int words(int s) {
    const int w = s == 0 ? E0 * pitch(0) : (strips(s - 1) * R - 1) * pitch(s) + ec(s - 1);
    const int r = s == K ? M * pitch(K) + M + 1 : (strips(s) * R + 1) * pitch(s) + width(s) + 2;
    return w > r ? w : r;
  }
  // array stride of each buffer: the largest of its layouts
  static constexpr int stride(int b) {
    int m = 0;
    for (int s = b; s <= K; s += 2) m = words(s) > m ? words(s) : m;
    return m;
  }
  // blocks of NT threads per CU that LDS of `words` words admits, at most
  // 16 waves per CU
  static constexpr int fit(int words, int nt) {
    const int b = (160 * 1024) / (words * int(sizeof(T)));
    const int w = 1024 / nt;
    return b < 1 ? 1 : (b < w ? b : w);
  }
  // Two layouts of the buffers: one stride for all eight arrays (E0 + R
  // rows of the widest pitch), or each buffer sized to the words its
  // layouts touch.  The per-buffer sizes cost the steps some address
  // arithmetic (about 8% at K = 8, 1024 threads), so they are used only
  // where they let more blocks share a CU, or where one stride would not
  // fit in LDS at all.
  static constexpr int max_words() {
    int m = (E0 + R) * max_pitch();
    for (int s = 0; s <= K; ++s) m = words(s) > m ? words(s) : m;
    return m;
  }
  static constexpr int UNI = max_words();
  static constexpr bool tight(int nt) {
    return fit(4 * (stride(0) + stride(1)), nt) > fit(8 * UNI, nt) || 8 * UNI * int(sizeof(T)) > 160 * 1024;
  }
  static_assert(valid(), "no bank-aligned pitch");
  // the plan as plain numbers, so that a step indexes constants
  struct Table {
    int pitch[K + 1], width[K];
  };
  static constexpr Table table() {
    Table t{};
    for (int s = 0; s <= K; ++s) t.pitch[s] = pitch(s);
    for (int s = 0; s < K; ++s) t.width[s] = width(s);
    return t;
  }
};

// Buffer geometry of the upwind level advance for a block of NT threads:
// array strides AS0 and AS1 of buffers 0 and 1 (buffer 1 starts at 4 AS0),
// and the blocks per CU the launch bounds ask for.  On large grids a second
// resident block overlaps one block's gather and write-back with another's
// steps.
// Rows per strip of the upwind level advance: as StripRows, for its first
// region of side M + K, except that 1024-thread blocks take at most 2 rows.
// Their first steps at large K then need a second, partial pass over the
// region, which costs less than 3-row strips in every step (K = 16, m = 32:
// 21.8 -> 19.5 us per launch).
template <int M, int K, int NT>
struct UpStripRows {
  static constexpr int EC0 = M + K;
  static constexpr int S = NT / EC0 > 0 ? NT / EC0 : 1;
  static constexpr int R0 = (EC0 + S - 1) / S;
  static constexpr int value = NT >= 1024 && R0 > 2 ? 2 : (R0 > 6 ? 6 : R0);
};

template <typename T, int M, int K, int NT>
struct UpGeom {
  static constexpr int R = UpStripRows<M, K, NT>::value;
  using P = UpPlan<T, M, K, R>;
  static constexpr bool TIGHT = P::tight(NT);
  static constexpr int AS0 = TIGHT ? P::stride(0) : P::UNI;
  static constexpr int AS1 = TIGHT ? P::stride(1) : P::UNI;
  static constexpr int WORDS = 4 * (AS0 + AS1);
  static constexpr int OCC = P::fit(WORDS, NT);
  // The last step stores to the output instead of to layout K: one barrier
  // and one LDS round trip fewer, 1-9% faster (FP64: 2-9% once 18 of its
  // weights are held in vector registers; with the weights parked in vector
  // lanes it had been 10-40% slower).  The 768-thread FP32 shape needs more
  // registers with it (96 instead of 80) and then no longer fits two blocks
  // per CU.
  static constexpr bool DIRECT = NT != 768;
  static_assert(AS0 >= P::stride(0) && AS1 >= P::stride(1), "buffer smaller than a layout");
};

template <typename T, int M, int K, int NT>
struct UpLds {
  T q[UpGeom<T, M, K, NT>::WORDS];  // buffer 0 then 1, each: average, corner, x-edge, y-edge
};

template <typename T, int M, int K, int NT>
__global__ __launch_bounds__(NT, (UpGeom<T, M, K, NT>::OCC)) void k_level_advance_up(const AdvanceArgs<T> A,
                                                                                   const AdvWeights<T> W) {
  constexpr int R = UpStripRows<M, K, NT>::value;
  using P = UpPlan<T, M, K, R>;
  constexpr int E0 = P::E0;
  constexpr int AS0 = UpGeom<T, M, K, NT>::AS0, AS1 = UpGeom<T, M, K, NT>::AS1;  // array strides of the buffers
  constexpr typename P::Table kTab = P::table();
  __shared__ UpLds<T, M, K, NT> S;

  const int pl = xcd_patch(int(blockIdx.x), int(gridDim.x));
  const int patch = A.first + pl;
  const int pix = pl % A.nx, piy = pl / A.nx;
  const size_t plane = size_t(M + 5) * A.pitch;

  // The 52 weights of a step (27 node, 25 average) stay in vector registers
  // for the whole launch (FP32; 52 of the 128 registers a lane has at this
  // occupancy).  Held as kernel arguments they overflow the scalar registers,
  // and every reload is a scalar load whose wait also drains all outstanding
  // LDS loads.  FP64 blocks of 512 or more threads have room for the 18
  // weights of the corner and x-edge stencils (36 registers); the other 34
  // then fit in scalar registers.  Without them the compiler parked FP64
  // weights in vector lanes, 48 lane moves per step beside 96 FMAs.  (The
  // 256-thread FP64 shapes got slower with them.)  The empty asm statements
  // only pin the register class.
  T wf[3][9], wq[25];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      wf[k][e] = W.w[k][1][e];
      if (sizeof(T) == 4 || (k < 2 && NT >= 512)) asm volatile("" : "+v"(wf[k][e]));
    }
#pragma unroll
  for (int e = 0; e < 25; ++e) {
    wq[e] = W.up_avg[e];
    if constexpr (sizeof(T) == 4) asm volatile("" : "+v"(wq[e]));
  }

  // ---- gather into layout 0: position (r, c) of the E0 x E0 block holds
  // local index (c - K, r - K); one source offset serves the four kinds
  {
    constexpr int EE = E0 * E0;
    constexpr int P0 = kTab.pitch[0];
    T* const g0 = &S.q[0];
    constexpr int NP = (EE + NT - 1) / NT;
    T v[NP][4];
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      const int e = int(threadIdx.x) + u * NT;
      if (u + 1 < NP || EE % NT == 0 || e < EE) {
        const int rr = e / E0, x = e - rr * E0;
        const int j = rr - K, i = x - K;
        const int oy = j < 0 ? -1 : (j >= M ? 1 : 0);
        const int ox = i < 0 ? -1 : (i >= M ? 1 : 0);
        const int src = level_nbr(A, pix, piy, ox, oy);
        const size_t off = size_t(src) * plane + size_t(j - oy * M + kGhost) * A.pitch + (i - ox * M + kGhost);
#pragma unroll
        for (int kind = 0; kind < 4; ++kind) v[u][kind] = A.in[kind][off];
      }
    }
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      const int e = int(threadIdx.x) + u * NT;
      if (u + 1 < NP || EE % NT == 0 || e < EE) {
        const int rr = e / E0, x = e - rr * E0;
        const int idx = rr * P0 + x;
#pragma unroll
        for (int kind = 0; kind < 4; ++kind) g0[kind * AS0 + idx] = v[u][kind];
      }
    }
  }
  __syncthreads();

#pragma unroll
  for (int s = 0; s < K; ++s) {
    const T* const qo = &S.q[(s & 1) ? 4 * AS0 : 0];
    T* const qn = &S.q[(s & 1) ? 0 : 4 * AS0];
    const int AI = (s & 1) ? AS1 : AS0;  // array stride of the buffer read
    const int AO = (s & 1) ? AS0 : AS1;  // and of the buffer written
    const int EC = P::ec(s);                 // region side; the region starts at column and row 1 of layout s
    const int WS = kTab.width[s];            // tasks per strip (columns past EC idle)
    const int PI = kTab.pitch[s];            // pitch of the layout read
    const int PO = kTab.pitch[s + 1];        // pitch of the layout written (origin one cell further in)
    const int ns = (EC + R - 1) / R;
    const int ntask = WS * ns;
    // task t -> column t % WS, strip t / WS; the window holds rows
    // [q R, q R + R + 1] and columns [c, c + 2] of every array of layout s
#pragma unroll 1
    for (int t0 = 0; t0 + int(threadIdx.x & ~63u) < ntask; t0 += NT) {  // wave-uniform
      const int t = t0 + int(threadIdx.x);
      const bool live = t < ntask;
      const int q = live ? t / WS : 0;
      const int ci = live ? t - q * WS : 0;
      const bool tok = live && ci < EC;  // columns EC..WS-1 load in bounds and store nothing
      const int br = q * R * PI + ci;
      const int bw = q * R * PO + ci;
      // One base offset per array, opaque to the compiler: an array's window
      // then lies within the 255-element offset range of paired LDS loads
      // from that base.  Folded into one base with large constants, the
      // loads were paired by column, with an address computed per pair.
      int ob[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        ob[k] = int(qo - &S.q[0]) + k * AI + br;
        asm("" : "+v"(ob[k]));
      }
      T wa[R + 2][3], w0[R + 2][3], w1[R + 2][3], w2[R + 2][3];
#pragma unroll
      for (int rr = 0; rr < R + 2; ++rr)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
          const int o = rr * PI + cc;
          wa[rr][cc] = S.q[ob[0] + o];
          w0[rr][cc] = S.q[ob[1] + o];
          w1[rr][cc] = S.q[ob[2] + o];
          w2[rr][cc] = S.q[ob[3] + o];
        }
#pragma unroll
      for (int u = 0; u < R; ++u) {
        // new node values at t + dt from the upwind source cells
        T f[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const int wr = u + 1 + up_off(k, 1), wc = 1 + up_off(k, 0);
          const T d[9] = {wa[wr][wc],     w0[wr][wc],     w0[wr][wc + 1], w0[wr + 1][wc], w0[wr + 1][wc + 1],
                          w1[wr][wc],     w1[wr][wc + 1], w2[wr][wc],     w2[wr + 1][wc]};
          T v = wf[k][0] * d[0];
#pragma unroll
          for (int e = 1; e < 9; ++e) v += wf[k][e] * d[e];
          f[k] = v;
        }
        // new average: the 25 old DOFs of the source cells (-1..0)^2
        T avg = T(0);
#pragma unroll
        for (int dj = -1; dj <= 0; ++dj)
#pragma unroll
          for (int di = -1; di <= 0; ++di) avg += wq[kUpA + (dj + 1) * 2 + (di + 1)] * wa[u + 1 + dj][1 + di];
#pragma unroll
        for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
          for (int di = -1; di <= 1; ++di) avg += wq[kUpC + (dj + 1) * 3 + (di + 1)] * w0[u + 1 + dj][1 + di];
#pragma unroll
        for (int dj = -1; dj <= 0; ++dj)
#pragma unroll
          for (int di = -1; di <= 1; ++di) avg += wq[kUpX + (dj + 1) * 3 + (di + 1)] * w1[u + 1 + dj][1 + di];
#pragma unroll
        for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
          for (int di = -1; di <= 0; ++di) avg += wq[kUpY + (dj + 1) * 2 + (di + 1)] * w2[u + 1 + dj][1 + di];
        if (s + 1 < K || !UpGeom<T, M, K, NT>::DIRECT) {
          if (tok) {  // strips past the region store into rows no later read touches
            const int idx = bw + u * PO;
            qn[idx] = avg;
            qn[AO + idx] = f[0];
            qn[2 * AO + idx] = f[1];
            qn[3 * AO + idx] = f[2];
          }
        } else {
          // the last step's region is the closed square of local cells
          // 0..M: store the interior averages and the closed-square nodes
          // straight to the output
          const int i = ci, j = q * R + u;
          if (tok && j <= M) {
            const size_t g = size_t(patch) * plane + size_t(j + kGhost) * A.pitch + (i + kGhost);
            A.out[1][g] = f[0];
            if (j < M) A.out[2][g] = f[1];
            if (i < M) A.out[3][g] = f[2];
            if (i < M && j < M) A.out[0][g] = avg;
          }
        }
      }
    }
    if (s + 1 < K || !UpGeom<T, M, K, NT>::DIRECT) __syncthreads();
  }

  // ---- write the interior averages and the closed-square nodes (layout K:
  // local cell (i, j) at row j, column i)
  if constexpr (!UpGeom<T, M, K, NT>::DIRECT) {
    constexpr int PK = kTab.pitch[K];
    constexpr int AF = (K & 1) ? AS1 : AS0;
    const T* const qf = &S.q[(K & 1) ? 4 * AS0 : 0];
    for (Walk2 w(threadIdx.x, NT, M + 1); w.y < M + 1; w.next()) {
      const int i = w.x, j = w.y;
      const int idx = j * PK + i;
      const size_t g = size_t(patch) * plane + size_t(j + kGhost) * A.pitch + (i + kGhost);
      A.out[1][g] = qf[AF + idx];
      if (j < M) A.out[2][g] = qf[2 * AF + idx];
      if (i < M) A.out[3][g] = qf[3 * AF + idx];
      if (i < M && j < M) A.out[0][g] = qf[idx];
    }
  }
}

// ---------------------------------------------------------------------------
// Common helpers for ghost fill and transfers.
// ---------------------------------------------------------------------------

template <typename T>
struct Bufs {
  T* p[2][4];
  int32_t npatch, pitch, m, ncomp;
  uint32_t mask;  // bit l: buffer of level l
};

template <typename T>
__device__ __forceinline__ T* buf_of(const Bufs<T>& B, int level, int kind) {
  return B.p[(B.mask >> level) & 1u][kind];
}

template <typename T>
__device__ __forceinline__ size_t at(const Bufs<T>& B, int comp, int patch, int i, int j) {
  return ((size_t(comp) * B.npatch + patch) * (B.m + 5) + size_t(j + kGhost)) * B.pitch + (i + kGhost);
}

__device__ __forceinline__ long long fdiv(long long a, long long b) {
  long long q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return q;
}

__device__ __forceinline__ int lut_find(const HierDev& H, int l, long long px, long long py) {
  if (l < 0 || l > H.lmax) return -1;
  const long long nx = (long long)H.npx0 << l, ny = (long long)H.npy0 << l;
  px = ((px % nx) + nx) % nx;
  py = ((py % ny) + ny) % ny;
  return H.lut[H.lut_off[l] + py * nx + px];
}

__device__ __forceinline__ double lagr(int a, double s) {
  return a < 0 ? 0.5 * s * (s - 1.0) : (a == 0 ? 1.0 - s * s : 0.5 * s * (s + 1.0));
}

// Reconstruction of cell (ci,cj) of leaf `patch` evaluated at reference
// point (xi, eta) (Sec. 2, eq. poly), in double precision.
template <typename T>
__device__ double eval_cell(const Bufs<T>& B, int level, int comp, int patch, int ci, int cj, double xi,
                            double eta) {
  const T* av = buf_of(B, level, 0);
  const T* co = buf_of(B, level, 1);
  const T* xe = buf_of(B, level, 2);
  const T* ye = buf_of(B, level, 3);
  double q[3][3];
  q[0][0] = co[at(B, comp, patch, ci, cj)];
  q[2][0] = co[at(B, comp, patch, ci + 1, cj)];
  q[0][2] = co[at(B, comp, patch, ci, cj + 1)];
  q[2][2] = co[at(B, comp, patch, ci + 1, cj + 1)];
  q[0][1] = xe[at(B, comp, patch, ci, cj)];
  q[2][1] = xe[at(B, comp, patch, ci + 1, cj)];
  q[1][0] = ye[at(B, comp, patch, ci, cj)];
  q[1][2] = ye[at(B, comp, patch, ci, cj + 1)];
  const double avg = av[at(B, comp, patch, ci, cj)];
  q[1][1] = (36.0 * avg - (q[0][0] + q[2][0] + q[0][2] + q[2][2]) - 4.0 * (q[0][1] + q[2][1] + q[1][0] + q[1][2])) / 16.0;
  double s = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double la = lagr(a - 1, xi);
#pragma unroll
    for (int b = 0; b < 3; ++b) s += q[a][b] * la * lagr(b - 1, eta);
  }
  return s;
}

// Simpson 3x3 average over the sub-square [xa, xa+1] x [ya, ya+1] of a cell's
// reference square (exact for the biquadratic reconstruction, Sec. 3.1).
template <typename T>
__device__ double quarter_avg(const Bufs<T>& B, int level, int comp, int patch, int ci, int cj, double xa,
                              double ya) {
  const double w[3] = {1.0, 4.0, 1.0};
  double s = 0.0;
#pragma unroll
  for (int p = 0; p < 3; ++p)
#pragma unroll
    for (int q = 0; q < 3; ++q)
      s += w[p] * w[q] * eval_cell(B, level, comp, patch, ci, cj, xa + 0.5 * p, ya + 0.5 * q);
  return s / 36.0;
}

// ---------------------------------------------------------------------------
// Ghost fill (Sec. 3.1, 3.2).  entries: packed (kind << 24) | ((i+2) << 12) |
// (j+2) for every DOF of the fill set of a patch.
//
// The source of each fill-set DOF depends only on the leaf set and on the
// lowest level allowed to serve as a source, so it is resolved once per
// hierarchy (k_fill_plan) into an op; every fill then applies the ops
// (k_fill_apply).  Phase 0 applies same-level and finer sources, phase 1
// (after it, since a coarse reconstruction reads nodes that phase 0 may
// rewrite on coarse-fine lines) the coarser ones.
// ---------------------------------------------------------------------------

// Source of fill-set DOF `code` of leaf t: averages from the same level, else
// the mean of four finer averages, else the Simpson average of the coarser
// reconstruction over the covered quarter; nodes from the finest leaf whose
// closed square holds them (candidates of one level in the order (hi,hi),
// (lo,hi), (hi,lo), (lo,lo)), the coarser reconstruction last.  Sources
// below level smin are not used; a DOF with no source keeps its value.
__device__ int4 fill_resolve(const HierDev& H, int m, int smin, int t, int32_t code) {
  const int4 none = make_int4(-1, 0, 0, 0);
  const int kind = code >> 24, i = ((code >> 12) & 0xfff) - kGhost, j = (code & 0xfff) - kGhost;
  const int lt = H.plevel[t];
  const long long I = (long long)H.pix[t] * m + i, J = (long long)H.piy[t] * m + j;
  if (kind == 0) {
    int src = -1, rel = 0;
    if (lt >= smin) src = lut_find(H, lt, fdiv(I, m), fdiv(J, m));
    if (src < 0 && lt + 1 <= H.lmax && lt + 1 >= smin) {
      src = lut_find(H, lt + 1, fdiv(2 * I, m), fdiv(2 * J, m));
      rel = 1;
    }
    if (src < 0 && lt - 1 >= 0 && lt - 1 >= smin) {
      src = lut_find(H, lt - 1, fdiv(I, 2 * m), fdiv(J, 2 * m));
      rel = -1;
    }
    if (src < 0) return none;
    if (rel == 0)
      return make_int4(src, fill_info(FO_COPY, 0, lt, 0, 0), int(I - fdiv(I, m) * m), int(J - fdiv(J, m) * m));
    if (rel == 1)
      return make_int4(src, fill_info(FO_MEAN4, 0, lt + 1, 0, 0), int(2 * I - fdiv(2 * I, m) * m),
                       int(2 * J - fdiv(2 * J, m) * m));
    const long long CI = fdiv(I, 2), CJ = fdiv(J, 2);
    const int qx = (I - 2 * CI == 0) ? 0 : 1, qy = (J - 2 * CJ == 0) ? 0 : 1;
    return make_int4(src, fill_info(FO_QAVG, 0, lt - 1, kFillPoints + qx + 2 * qy, 1), int(CI - fdiv(CI, m) * m),
                     int(CJ - fdiv(CJ, m) * m));
  }
  // node position in level-(lt+1) half-cell units
  const long long FX = 4 * I + (kind == 3 ? 2 : 0);
  const long long FY = 4 * J + (kind == 2 ? 2 : 0);
  int src = -1, rel = 0, sh = 0;
  long long sx = 0, sy = 0;  // source-local position in level-(lt+1) half-cell units
  for (int k = lt + 1; k >= lt - 1 && src < 0; --k) {
    if (k < 0 || k > H.lmax || k < smin) continue;
    sh = lt + 1 - k;
    const long long P = 2LL * m << sh;
    const long long hx = fdiv(FX, P), hy = fdiv(FY, P);
    const bool bx = (FX - hx * P) == 0, by = (FY - hy * P) == 0;
    const int ox[4] = {0, 1, 0, 1}, oy[4] = {0, 0, 1, 1};
    for (int o = 0; o < 4; ++o) {
      if (ox[o] && !bx) continue;
      if (oy[o] && !by) continue;
      const int id = lut_find(H, k, hx - ox[o], hy - oy[o]);
      if (id < 0) continue;
      src = id;
      rel = k - lt;
      sx = FX - (hx - ox[o]) * P;
      sy = FY - (hy - oy[o]) * P;
      break;
    }
  }
  if (src < 0) return none;
  const long long unit = 1LL << sh;
  if (rel >= 0) {
    const long long X = sx / unit, Y = sy / unit;  // source half-cell units
    if (rel == 0 && src == t) {
      // the target itself: keep unless the match is a periodic image
      const long long Xt = 2 * i + (kind == 3 ? 1 : 0), Yt = 2 * j + (kind == 2 ? 1 : 0);
      if (X == Xt && Y == Yt) return none;
    }
    const int ls = lt + rel;
    const bool ex = (X % 2) == 0, ey = (Y % 2) == 0;
    if (ex && ey) return make_int4(src, fill_info(FO_COPY, 1, ls, 0, 0), int(X / 2), int(Y / 2));
    if (ex) return make_int4(src, fill_info(FO_COPY, 2, ls, 0, 0), int(X / 2), int((Y - 1) / 2));
    return make_int4(src, fill_info(FO_COPY, 3, ls, 0, 0), int((X - 1) / 2), int(Y / 2));
  }
  // coarser: reconstruction of the covering cell at a quarter-step point
  // (sx, sy are multiples of 2: fine nodes sit on a half-of-half-cell grid)
  const long long cx2 = sx / 2, cy2 = sy / 2;  // coarse quarter-cell units
  int ci = int(cx2 / 4), cj = int(cy2 / 4);
  ci = min(max(ci, 0), m - 1);
  cj = min(max(cj, 0), m - 1);
  const int px = int(cx2 - 4LL * ci), py = int(cy2 - 4LL * cj);  // 0..4: xi = px/2 - 1
  return make_int4(src, fill_info(FO_EVAL, 0, lt - 1, px + 5 * py, 1), ci, cj);
}

// Direction d = (oy + 1) * 3 + (ox + 1) of block position (i, j) of a patch
// (ox = -1, 0, 1 for i < 0, 0 <= i < m, i >= m; oy likewise): the patch
// whose interior holds it on a complete level.
__device__ __forceinline__ int gather_dir(int i, int j, int m) {
  const int ox = i < 0 ? -1 : (i >= m ? 1 : 0), oy = j < 0 ? -1 : (j >= m ? 1 : 0);
  return (oy + 1) * 3 + (ox + 1);
}

// One block per leaf: the plan row of the leaf and a flag word (bit p: the
// leaf has ops of phase p).  With nbr (the plan of smin = 0), also the
// leaf's same-level neighbours nbr[t][d] (-1 where the direction holds no
// leaf of its level; d = 4 is the leaf) and gnflags[t] bit d: every fill-set
// DOF in direction d resolves to the copy a same-level gather would read
// (the neighbour's own DOF at the shifted position; for d = 4, the leaf's
// own value).  Such ops resolve the same way for every source bound up to
// the leaf's level, since same-level and finer sources are then admissible.
__global__ __launch_bounds__(kThreads) void k_fill_plan(const HierDev H, const int32_t* entries, int nentries, int m,
                                                        int smin, int4* plan, uint32_t* flags, int32_t* nbr,
                                                        uint32_t* gnflags) {
  const int t = blockIdx.x;
  const int lt = H.plevel[t];
  __shared__ int32_t nb[9];
  __shared__ uint32_t gn;
  if (nbr) {
    if (threadIdx.x < 9) {
      const int d = threadIdx.x, ox = d % 3 - 1, oy = d / 3 - 1;
      nb[d] = d == 4 ? t : lut_find(H, lt, (long long)H.pix[t] + ox, (long long)H.piy[t] + oy);
      nbr[size_t(t) * 9 + d] = nb[d];
    }
    if (threadIdx.x == 0) gn = 0x1ffu;
    __syncthreads();
  }
  int has0 = 0, has1 = 0;
  for (int e = threadIdx.x; e < nentries; e += kThreads) {
    const int4 op = fill_resolve(H, m, smin, t, entries[e]);
    plan[size_t(t) * nentries + e] = op;
    if (op.x >= 0) {
      if ((op.y >> 16) & 1) has1 = 1;
      else has0 = 1;
    }
    if (nbr) {
      const int32_t code = entries[e];
      const int kind = code >> 24, i = ((code >> 12) & 0xfff) - kGhost, j = (code & 0xfff) - kGhost;
      const int d = gather_dir(i, j, m), ox = d % 3 - 1, oy = d / 3 - 1;
      bool ok;
      if (d == 4) {
        ok = op.x < 0;
      } else {
        const int fo = op.y & 3, skind = (op.y >> 2) & 3, ls = (op.y >> 4) & 15;
        ok = nb[d] >= 0 && op.x == nb[d] && fo == FO_COPY && skind == kind && ls == lt && op.z == i - ox * m &&
             op.w == j - oy * m;
      }
      if (!ok) atomicAnd(&gn, ~(1u << d));
    }
  }
  has0 = __syncthreads_or(has0);
  has1 = __syncthreads_or(has1);
  if (threadIdx.x == 0) {
    flags[t] = uint32_t(has0) | (uint32_t(has1) << 1);
    if (nbr) gnflags[t] = gn;
  }
}

template <typename T>
struct FillArgs {
  Bufs<T> B;
  const int32_t* plevel;
  const int32_t* entries;
  const int4* plan;
  const uint32_t* flags;
  const FillWeights* W;
  int32_t nentries, chunks, first_target, phase;
};

template <typename T>
__global__ __launch_bounds__(kThreads) void k_fill_apply(const FillArgs<T> A) {
  const int w = xcd_patch(int(blockIdx.x), int(gridDim.x));
  const int tl = w / A.chunks;
  const int chunk = w - tl * A.chunks;
  const int t = A.first_target + tl;
  if (!((A.flags[t] >> A.phase) & 1u)) return;  // block-uniform
  const Bufs<T>& B = A.B;
  const int lt = A.plevel[t], nc = B.ncomp;
  const size_t cstride = size_t(B.npatch) * (B.m + 5) * B.pitch;  // component stride
  for (int e = chunk * kThreads + threadIdx.x; e < A.nentries; e += A.chunks * kThreads) {
    const int4 op = A.plan[size_t(t) * A.nentries + e];
    if (op.x < 0 || ((op.y >> 16) & 1) != A.phase) continue;
    const int32_t code = A.entries[e];
    const int kind = code >> 24, i = ((code >> 12) & 0xfff) - kGhost, j = (code & 0xfff) - kGhost;
    const int fo = op.y & 3, skind = (op.y >> 2) & 3, ls = (op.y >> 4) & 15, pos = (op.y >> 8) & 255;
    T* const dst = buf_of(B, lt, kind) + at(B, 0, t, i, j);
    if (fo == FO_COPY) {
      const T* s = buf_of(B, ls, skind) + at(B, 0, op.x, op.z, op.w);
      for (int q = 0; q < nc; ++q) dst[q * cstride] = s[q * cstride];
    } else if (fo == FO_MEAN4) {
      // mean of the four fine averages (fine -> coarse transfer)
      const T* s = buf_of(B, ls, 0) + at(B, 0, op.x, op.z, op.w);
      const int P = B.pitch;
      for (int q = 0; q < nc; ++q) {
        const T* v = s + q * cstride;
        dst[q * cstride] = T(0.25 * ((double(v[0]) + double(v[1])) + (double(v[P]) + double(v[P + 1]))));
      }
    } else {
      // coarse reconstruction: point value (EVAL) or quarter average (QAVG)
      const double* w = A.W->w[pos];
      const int P = B.pitch;
      const size_t o = at(B, 0, op.x, op.z, op.w);
      const T* av = buf_of(B, ls, 0) + o;
      const T* co = buf_of(B, ls, 1) + o;
      const T* xe = buf_of(B, ls, 2) + o;
      const T* ye = buf_of(B, ls, 3) + o;
      for (int q = 0; q < nc; ++q) {
        const size_t c = q * cstride;
        double v = w[0] * double(av[c]);
        v += w[1] * double(co[c]);
        v += w[2] * double(co[c + 1]);
        v += w[3] * double(co[c + P]);
        v += w[4] * double(co[c + P + 1]);
        v += w[5] * double(xe[c]);
        v += w[6] * double(xe[c + 1]);
        v += w[7] * double(ye[c]);
        v += w[8] * double(ye[c + P]);
        dst[c] = T(v);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Batched subcycled coarse step (Sec. 3.2) for the constant-coefficient
// equations: one launch per substep start time steps every patch of every
// level that starts a step then.
//
// With the finest level F and time points tau = 0 .. 2^F - 1 in units of the
// finest step, level l starts a step at tau when 2^(F-l) divides tau; the
// coarsest such level is l0(tau).  The recursion of Sec. 3.2 fills levels >=
// l0 from sources of level >= l0 just before those steps, and the steps read
// only their own patch and its halo, so all of them can share a launch.  The
// halo is not filled in HBM: k_amr_step stages every fill-set DOF straight
// from the source the fill plan of that time point names (same-level copy,
// mean of four finer averages, coarser reconstruction), the values a fill
// would have written.  A coarser reconstruction reads the source leaf's
// closed-square nodes, whose copies on coarse-fine lines the fill makes equal
// to the finer leaf's vertices first (the second fill phase); k_amr_sync does
// that copy, together with the conservative fix of the levels that just
// completed a pair of fine substeps, before the launch.
//
// With fused pairs the launches are those of the even time points, and the
// finest level's block there also takes the odd time point's substep (see
// the pair branch of k_amr_step).
// ---------------------------------------------------------------------------

template <typename T>
struct AmrStepArgs {
  T* p[2][4];                      // the two state buffers
  int32_t npatch, pitch;
  uint32_t mask;                   // level l's data before the step: p[(mask >> l) & 1]
  int32_t nlev, lev0;              // levels lev0 .. lev0 + nlev - 1 step
  int32_t first[kMaxLevels];       // first leaf of each of those levels
  int32_t bstart[kMaxLevels + 1];  // first block of range kk, level nlev - 1 - kk (multiples of 8); bstart[nlev] = blocks
  int32_t items[kMaxLevels];       // (patch, tile) items of each level, <= its block range
  int32_t region[kMaxLevels], tiles[kMaxLevels], rows[kMaxLevels];
  double len_dt_x[kMaxLevels], len_dt_y[kMaxLevels];
  T dtdx, dtdy, a, b, c;
  double* reg;                     // FP64 flux registers
  const uint8_t* side_mask;
  const int4* plan;                // fill plan of this time point, [nleaves][nentries]
  const int32_t* entries;          // fill-set entries; the first ninner lie within one cell of the interior
  int32_t nentries, ninner;
  const FillWeights* fw;
  const int32_t* nbr;              // [nleaves][9] same-level neighbours (k_fill_plan)
  const uint32_t* gnflags;         // [nleaves] directions staged by the same-level gather
  int32_t pair;                    // the last level takes both substeps of its pair
};

// Interior DOFs of a patch that no fill writes (af_ctx_create's fill set is
// the complement): averages of cells [0,m)^2 and nodes strictly inside.
__device__ __forceinline__ bool own_dof(int kind, int i, int j, int m) {
  switch (kind) {
    case 0: return i >= 0 && i < m && j >= 0 && j < m;
    case 1: return i >= 1 && i <= m - 1 && j >= 1 && j <= m - 1;
    case 2: return i >= 1 && i <= m - 1 && j >= 0 && j <= m - 1;
    default: return i >= 0 && i <= m - 1 && j >= 1 && j <= m - 1;
  }
}

// Value of fill-set DOF (kind, i, j) of leaf t as the fill plan resolves it
// (op), component q; own = the leaf's own buffer (for "no source: keep").
template <typename T>
__device__ __forceinline__ T planned_value(T* const (&p)[2][4], uint32_t mask, int npatch, int pitch, int m,
                                           const FillWeights* fw, const int4& op, const T* own, int q) {
  const size_t plane = size_t(m + 5) * pitch;
  if (op.x < 0) return own[size_t(q) * npatch * plane];
  const int fo = op.y & 3, skind = (op.y >> 2) & 3, ls = (op.y >> 4) & 15, pos = (op.y >> 8) & 255;
  T* const* sb = p[(mask >> ls) & 1u];
  const size_t o = (size_t(q) * npatch + op.x) * plane + size_t(op.w + kGhost) * pitch + (op.z + kGhost);
  if (fo == FO_COPY) return sb[skind][o];
  if (fo == FO_MEAN4) {
    const T* v = sb[0] + o;
    return T(0.25 * ((double(v[0]) + double(v[1])) + (double(v[pitch]) + double(v[pitch + 1]))));
  }
  const double* w = fw->w[pos];
  const T* av = sb[0] + o;
  const T* co = sb[1] + o;
  const T* xe = sb[2] + o;
  const T* ye = sb[3] + o;
  double v = w[0] * double(av[0]);
  v += w[1] * double(co[0]);
  v += w[2] * double(co[1]);
  v += w[3] * double(co[pitch]);
  v += w[4] * double(co[pitch + 1]);
  v += w[5] * double(xe[0]);
  v += w[6] * double(xe[1]);
  v += w[7] * double(ye[0]);
  v += w[8] * double(ye[pitch]);
  return T(v);
}

// The stencil weights a batched step reads: acoustics through wdev, the
// advection weights (the kernel argument) as they are.  As a kernel argument
// the acoustic table is loaded into scalar registers at entry, more than
// there are, and the compiler parked the rest in vector lanes (a quarter of
// the node phase's vector instructions were lane reads).  Through a
// read-only pointer argument each node kind's weights are scalar loads where
// the kind is evaluated.
template <typename T, int EQ>
__device__ __forceinline__ const typename WSel<T, EQ>::type& amr_weights(const AcOrbitWeights<T>* wdev,
                                                                        const typename WSel<T, EQ>::type& W) {
  if constexpr (EQ == 1)
    return *wdev;
  else
    return W;
}

template <typename T, int EQ, int M, int TY, bool PAIR>
__global__ __launch_bounds__(kThreads) void k_amr_step(const AmrStepArgs<T> A, const typename WSel<T, EQ>::type W,
                                                       const AcOrbitWeights<T>* __restrict__ wdev) {
  static_assert(EQ == 0 || EQ == 1, "constant-coefficient equations only");
  static_assert(!PAIR || TY >= M + 2, "a fused pair steps the whole layer-1 region in one block");
  constexpr int NCOMP = EQ == 1 ? 3 : 1;
  constexpr int NR = TY + 3;
  constexpr int NC = M + 5;
  __shared__ StepLds<T, NCOMP, NR, NC, kLdsAlias> L;

  // ---- block -> (level, patch, tile).  Each level's block range is a
  // multiple of 8 long, so every XCD takes an equal share of every level (the
  // coarse levels' blocks, which fill most of their halo from the plan, are
  // slow ones), and within a level a contiguous run of its leaves.  The
  // ranges run from the finest level (range kk = 0) to the coarsest: the
  // finest level's blocks, which carry both substeps of a fused pair, are
  // dispatched first, and the shorter ones fill the end of the launch.
  const int b = int(blockIdx.x);
  int kk = 0;
  while (kk + 1 < A.nlev && b >= A.bstart[kk + 1]) ++kk;
  const int k = A.nlev - 1 - kk;
  const int lvl = A.lev0 + k;
  const int local = xcd_patch(b - A.bstart[kk], A.bstart[kk + 1] - A.bstart[kk]);
  if (local >= A.items[k]) return;  // padding of the level's range (block-uniform)
  const int tiles = A.tiles[k], rows = A.rows[k], region = A.region[k];
  const int pl = local / tiles;
  const int tile = local - pl * tiles;
  const int patch = A.first[k] + pl;
  const int ilo = -region, ihi = M + region;
  const int jlo = ilo + tile * rows;
  const int jhi = min(jlo + rows, ihi);
  if (jlo >= jhi) return;  // block-uniform; cannot happen for the compiled (m, TY) pairs
  const int cur = (A.mask >> lvl) & 1;
  const size_t plane = size_t(M + 5) * A.pitch;
  const T* const* in = A.p[cur];

  // ---- stage rows jlo-1 .. jlo-1+NR-1 (those up to m+2) of the patch
  // block.  Pass A: the DOFs no fill writes from the patch itself, and the
  // fill-set DOFs of every direction whose planned sources are the same-level
  // gather's (gnflags) from the neighbour's interior; all loads of a thread
  // are issued before its stores.  Pass B: the other fill-set DOFs from the
  // plan.  An interior-region step reads only cells [-1, m] and nodes
  // [-1, m+1], so both passes skip the outer ring then.
  const uint32_t gn = A.gnflags[patch];
  const int32_t* const nbrow = A.nbr + size_t(patch) * 9;
  const int lo = region == 0 ? -1 : -2, hi = M + 2 - (region == 0 ? 1 : 0);
  {
    constexpr int PE = NR * NC;
    constexpr int PER = (PE + kThreads - 1) / kThreads;
    // element offsets fit in 32 bits (checked on the host): the loads take a
    // uniform plane base and a 32-bit per-lane offset
    const uint32_t plane32 = uint32_t(M + 5) * uint32_t(A.pitch);
    const uint32_t cstride = uint32_t(A.npatch) * plane32;
    uint32_t off[PER][4];
    uint32_t use = 0;  // bit 4u + kind: position u, kind loaded
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = int(threadIdx.x) + u * kThreads;
      const int rr = e / NC, x = e - rr * NC;
      const int j = jlo - 1 + rr, i = x - kGhost;
      const bool valid = e < PE && j <= hi && j >= lo && i >= lo && i <= hi;
      const int d = gather_dir(i, j, M), ox = d % 3 - 1, oy = d / 3 - 1;
      const bool gd = valid && ((gn >> d) & 1u);
      const int src = gd && d != 4 ? nbrow[d] : patch;
      const uint32_t o_own = uint32_t(patch) * plane32 + uint32_t(j + kGhost) * uint32_t(A.pitch) + uint32_t(x);
      const uint32_t o_src = uint32_t(src) * plane32 + uint32_t(j - oy * M + kGhost) * uint32_t(A.pitch) +
                             uint32_t(i - ox * M + kGhost);
#pragma unroll
      for (int kind = 0; kind < 4; ++kind) {
        const bool own = valid && own_dof(kind, i, j, M);
        off[u][kind] = own ? o_own : o_src;
        if (own || gd) use |= 1u << (4 * u + kind);
      }
    }
    T v[PER][4][NCOMP];
#pragma unroll
    for (int u = 0; u < PER; ++u)
#pragma unroll
      for (int kind = 0; kind < 4; ++kind)
        if ((use >> (4 * u + kind)) & 1u)
#pragma unroll
          for (int q = 0; q < NCOMP; ++q) v[u][kind][q] = in[kind][off[u][kind] + uint32_t(q) * cstride];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = int(threadIdx.x) + u * kThreads;
      const int rr = e / NC, x = e - rr * NC;
#pragma unroll
      for (int kind = 0; kind < 4; ++kind)
        if ((use >> (4 * u + kind)) & 1u)
#pragma unroll
          for (int q = 0; q < NCOMP; ++q) L.in[kind][q][rr][x] = v[u][kind][q];
    }
  }
  if (gn != 0x1ffu) {
    const int nent = region == 0 ? A.ninner : A.nentries;
    const int4* const prow = A.plan + size_t(patch) * A.nentries;
    for (int e = threadIdx.x; e < nent; e += kThreads) {
      const int32_t code = A.entries[e];
      const int kind = code >> 24, i = ((code >> 12) & 0xfff) - kGhost, j = (code & 0xfff) - kGhost;
      const int rr = j - (jlo - 1);
      if (rr < 0 || rr >= NR || ((gn >> gather_dir(i, j, M)) & 1u)) continue;
      const int4 op = prow[e];
      const T* own = in[kind] + size_t(patch) * plane + size_t(j + kGhost) * A.pitch + (i + kGhost);
#pragma unroll
      for (int q = 0; q < NCOMP; ++q)
        L.in[kind][q][rr][i + kGhost] = planned_value<T>(A.p, A.mask, A.npatch, A.pitch, M, A.fw, op, own, q);
    }
  }
  __syncthreads();

  StepIO<T> io;
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) io.out[kk] = A.p[cur ^ 1][kk];
  io.npatch = A.npatch;
  io.pitch = A.pitch;
  io.patch = patch;
  io.region = region;
  io.dtdx = A.dtdx;
  io.dtdy = A.dtdy;
  io.a = A.a;
  io.b = A.b;
  io.c = A.c;
  io.len_dt_x = A.len_dt_x[k];
  io.len_dt_y = A.len_dt_y[k];
  io.reg = (A.reg && A.side_mask) ? A.reg : nullptr;
  io.smask = io.reg ? A.side_mask[patch] : 0u;
  bool pair = false;
  if constexpr (PAIR) pair = A.pair && k == A.nlev - 1;
  if (pair) {
    // the finest level's pair of substeps (Sec. 3.2).  The first advances the
    // layer-1 region (cells [-1, m], nodes [-1, m+1]) into LDS; the second
    // steps the interior from exactly those values.  They are what a fill
    // would stage at the odd time point: the fill there has no coarser
    // sources, so coarse-fine ghosts keep the layer-1 values, and a
    // same-level neighbour's interior is the same arithmetic on the same
    // data.
    if constexpr (PAIR) {
      step_compute<T, EQ, M, TY, true>(L, io, amr_weights<T, EQ>(wdev, W), jlo, jhi, T(0), T(0));
      __syncthreads();
      io.region = 0;  // interior
      step_compute<T, EQ, M, TY>(L, io, amr_weights<T, EQ>(wdev, W), 0, M, T(0), T(0), -jlo);
    }
  } else {
    step_compute<T, EQ, M, TY>(L, io, amr_weights<T, EQ>(wdev, W), jlo, jhi, T(0), T(0));
  }
}

// Before the launch of a time point: the conservative fix (Sec. 3.2) of the
// coarse cells next to finer leaves, for the faces [0, nfaces) (the levels
// that just completed a pair of fine substeps), and the fill's copies of
// finer or same-level vertices onto the closed-square boundary nodes of the
// leaves canon[0 .. ncanon) (those with a neighbour of another level: a
// coarser reconstruction in the next launch may read their nodes).  The two
// touch disjoint DOFs: the fix only cell averages, the copies only nodes,
// read from leaves that own them (never a copy target).  Blocks [0, ncanon)
// copy, one per leaf; the rest fix.
template <typename T>
struct AmrSyncArgs {
  Bufs<T> B;
  const int32_t* plevel;
  const int4* cops;         // the vertex copies (k_canon_ops), ncops of them
  int32_t ncops;
  const CFFace* faces;
  int32_t nfaces;
  double* reg;
  double inv_area0;         // 1 / (dx_0 dy_0); level l: times 4^l
};

template <typename T>
__device__ void reflux_face_group(const Bufs<T>& B, const CFFace* faces, int nfaces, int f, double* reg,
                                  const int32_t* plevel, double inv_area0) {
  const int m = B.m, nc = B.ncomp;
  auto cell_of = [&](const CFFace& F, int* ci, int* cj) {
    *ci = F.side == 0 ? 0 : (F.side == 1 ? m - 1 : F.k);
    *cj = F.side == 2 ? 0 : (F.side == 3 ? m - 1 : F.k);
  };
  int ci, cj;
  cell_of(faces[f], &ci, &cj);
  if (f > 0) {
    int pi, pj;
    cell_of(faces[f - 1], &pi, &pj);
    if (faces[f - 1].coarse == faces[f].coarse && pi == ci && pj == cj) return;
  }
  const int level = plevel[faces[f].coarse];
  const double inv_area = inv_area0 * double(1LL << (2 * level));
  T* av = buf_of(B, level, 0);
  for (int g = f; g < nfaces; ++g) {
    const CFFace F = faces[g];
    int gi, gj;
    cell_of(F, &gi, &gj);
    if (F.coarse != faces[f].coarse || gi != ci || gj != cj) break;
    const double sgn = (F.side == 1 || F.side == 3) ? 1.0 : -1.0;
    const int opp = F.side ^ 1;
    double* Rc = reg + (size_t(F.coarse) * 4 + F.side) * m * nc + size_t(F.k) * nc;
    double* Rf = reg + (size_t(F.fine) * 4 + opp) * m * nc + size_t(F.fk) * nc;
    for (int q = 0; q < nc; ++q) {
      const double rf = Rf[q] + Rf[nc + q];
      const size_t idx = at(B, q, F.coarse, ci, cj);
      av[idx] = T(double(av[idx]) + sgn * (Rc[q] - rf) * inv_area);
      Rc[q] = 0.0;
      Rf[q] = 0.0;
      Rf[nc + q] = 0.0;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_amr_sync(const AmrSyncArgs<T> A) {
  const Bufs<T>& B = A.B;
  const int cblocks = (A.ncops + kThreads - 1) / kThreads;
  if (int(blockIdx.x) < cblocks) {
    const int e = int(blockIdx.x) * kThreads + int(threadIdx.x);
    if (e >= A.ncops) return;
    const int4 op = A.cops[e];
    if (op.x < 0) return;  // the leaf owns this node
    const int di = (op.z & 0xff) - kGhost, dj = ((op.z >> 8) & 0xff) - kGhost;
    const int kind = (op.z >> 16) & 3, lt = (op.z >> 20) & 15, skind = (op.z >> 24) & 3, ls = (op.z >> 28) & 15;
    const int si = (op.w & 0xffff) - kGhost, sj = (op.w >> 16) - kGhost;
    const size_t cstride = size_t(B.npatch) * (B.m + 5) * B.pitch;
    T* const dst = buf_of(B, lt, kind) + at(B, 0, op.x, di, dj);
    const T* const src = buf_of(B, ls, skind) + at(B, 0, op.y, si, sj);
    for (int q = 0; q < B.ncomp; ++q) dst[q * cstride] = src[q * cstride];
    return;
  }
  const int f = (int(blockIdx.x) - cblocks) * kThreads + int(threadIdx.x);
  if (f < A.nfaces) reflux_face_group(B, A.faces, A.nfaces, f, A.reg, A.plevel, A.inv_area0);
}

// The fill's vertex copies onto the closed-square boundary nodes of the
// leaves canon[0 .. ncanon), resolved once per hierarchy and source bound
// from the fill plan into ops[k * nbnd + b] (boundary entry b of leaf
// canon[k]): x = target leaf (-1: the leaf owns the node), y = source leaf,
// z = target column | row << 8 (both + kGhost) | kind << 16 | target level
// << 20 | source kind << 24 | source level << 28, w = source column |
// row << 16 (both + kGhost).  k_amr_sync then copies with one op load and
// one source load per node.
__global__ void k_canon_ops(const int4* plan, const int32_t* entries, int nentries, const int32_t* bnd, int nbnd,
                            const int32_t* canon, int ncanon, const int32_t* plevel, int4* ops) {
  const long n = long(ncanon) * nbnd;
  for (long e = blockIdx.x * long(blockDim.x) + threadIdx.x; e < n; e += long(gridDim.x) * blockDim.x) {
    const int k = int(e / nbnd), b = int(e - long(k) * nbnd);
    const int t = canon[k];
    const int ent = bnd[b];
    const int4 op = plan[size_t(t) * nentries + ent];
    int4 r = make_int4(-1, 0, 0, 0);
    if (op.x >= 0) {
      const int32_t code = entries[ent];
      const int kind = code >> 24, i = (code >> 12) & 0xfff, j = code & 0xfff;  // + kGhost
      const int skind = (op.y >> 2) & 3, ls = (op.y >> 4) & 15;
      r = make_int4(t, op.x, i | (j << 8) | (kind << 16) | (plevel[t] << 20) | (skind << 24) | (ls << 28),
                    (op.z + kGhost) | ((op.w + kGhost) << 16));
    }
    ops[e] = r;
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_flux_correct(Bufs<T> B, const CFFace* faces, int nfaces,
                                                           double* reg, int level, double inv_area) {
  const int f = blockIdx.x * kThreads + threadIdx.x;
  if (f >= nfaces) return;
  const int m = B.m, nc = B.ncomp;
  auto cell_of = [&](const CFFace& F, int* ci, int* cj) {
    *ci = F.side == 0 ? 0 : (F.side == 1 ? m - 1 : F.k);
    *cj = F.side == 2 ? 0 : (F.side == 3 ? m - 1 : F.k);
  };
  int ci, cj;
  cell_of(faces[f], &ci, &cj);
  if (f > 0) {
    int pi, pj;
    cell_of(faces[f - 1], &pi, &pj);
    if (faces[f - 1].coarse == faces[f].coarse && pi == ci && pj == cj) return;
  }
  T* av = buf_of(B, level, 0);
  for (int g = f; g < nfaces; ++g) {
    const CFFace F = faces[g];
    int gi, gj;
    cell_of(F, &gi, &gj);
    if (F.coarse != faces[f].coarse || gi != ci || gj != cj) break;
    const double sgn = (F.side == 1 || F.side == 3) ? 1.0 : -1.0;
    const int opp = F.side ^ 1;
    double* Rc = reg + (size_t(F.coarse) * 4 + F.side) * m * nc + size_t(F.k) * nc;
    double* Rf = reg + (size_t(F.fine) * 4 + opp) * m * nc + size_t(F.fk) * nc;
    for (int q = 0; q < nc; ++q) {
      const double rf = Rf[q] + Rf[nc + q];
      const size_t idx = at(B, q, F.coarse, ci, cj);
      av[idx] = T(double(av[idx]) + sgn * (Rc[q] - rf) * inv_area);
      Rc[q] = 0.0;
      Rf[q] = 0.0;
      Rf[nc + q] = 0.0;
    }
  }
}

// ---------------------------------------------------------------------------
// Tagging (Sec. 3; criteria of Sec. 4.1, 4.4): one block per leaf.
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(kThreads) void k_tag(Bufs<T> B, HierDev H, int mode, int comp, double inv2dx0,
                                                  double inv2dy0, double tr, double tc, int8_t* tags,
                                                  double* values) {
  const int p = blockIdx.x;
  const int l = H.plevel[p];
  const int m = B.m;
  const T* av = buf_of(B, l, 0);
  const double s2x = inv2dx0 * double(1 << l), s2y = inv2dy0 * double(1 << l);
  double vmax = -1e300, vmin = 1e300;
  for (int e = threadIdx.x; e < m * m; e += kThreads) {
    const int i = e % m, j = e / m;
    if (mode == 0) {
      const double gx = fabs(double(av[at(B, comp, p, i + 1, j)]) - double(av[at(B, comp, p, i - 1, j)])) * s2x;
      const double gy = fabs(double(av[at(B, comp, p, i, j + 1)]) - double(av[at(B, comp, p, i, j - 1)])) * s2y;
      vmax = fmax(vmax, fmax(gx, gy));
    } else {
      const double v = av[at(B, comp, p, i, j)];
      vmax = fmax(vmax, v);
      vmin = fmin(vmin, v);
    }
  }
  __shared__ double smax[kThreads], smin[kThreads];
  smax[threadIdx.x] = vmax;
  smin[threadIdx.x] = vmin;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double v = mode == 0 ? smax[0] : smax[0] - smin[0];
    int8_t tg = 0;
    if (v >= tr && l < H.lmax) tg = 1;
    else if (v < tc && l > 0) tg = -1;
    tags[p] = tg;
    if (values) values[p] = v;
  }
}

// ---------------------------------------------------------------------------
// Regrid transfer (Sec. 3.1): one block per new leaf.
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(kThreads) void k_transfer(Bufs<T> OLD, HierDev HO, Bufs<T> NEW, const Transfer* tr) {
  const int p = blockIdx.x;
  const Transfer X = tr[p];
  const int m = NEW.m, nc = NEW.ncomp;
  const int n_avg = m * m, n_c = (m + 1) * (m + 1), n_x = m * (m + 1), n_y = (m + 1) * m;
  const int total = n_avg + n_c + n_x + n_y;
  for (int e = threadIdx.x; e < total; e += kThreads) {
    int kind, i, j;
    if (e < n_avg) { kind = 0; i = e % m; j = e / m; }
    else if (e < n_avg + n_c) { const int f = e - n_avg; kind = 1; i = f % (m + 1); j = f / (m + 1); }
    else if (e < n_avg + n_c + n_x) { const int f = e - n_avg - n_c; kind = 2; i = f % (m + 1); j = f / (m + 1); }
    else { const int f = e - n_avg - n_c - n_x; kind = 3; i = f % m; j = f / m; }
    for (int q = 0; q < nc; ++q) {
      double val;
      if (X.mode == 0) {
        const int s = X.src[0];
        val = buf_of(OLD, HO.plevel[s], kind)[at(OLD, q, s, i, j)];
      } else if (X.mode == 1) {
        const int s = X.src[0];
        const int ls = HO.plevel[s];
        if (kind == 0) {
          const int fi = X.qx * m + i, fj = X.qy * m + j;
          val = quarter_avg(OLD, ls, q, s, fi >> 1, fj >> 1, (fi & 1) ? 0.0 : -1.0, (fj & 1) ? 0.0 : -1.0);
        } else {
          // node position in parent half-cell units
          double xs = double(X.qx * m + i), ys = double(X.qy * m + j);
          if (kind == 2) ys += 0.5;
          if (kind == 3) xs += 0.5;
          int ci = min(max(int(floor(xs / 2.0)), 0), m - 1), cj = min(max(int(floor(ys / 2.0)), 0), m - 1);
          val = eval_cell(OLD, ls, q, s, ci, cj, xs - (2.0 * ci + 1.0), ys - (2.0 * cj + 1.0));
        }
      } else {
        if (kind == 0) {
          const int fi = 2 * i, fj = 2 * j;
          const int qx = fi / m, qy = fj / m;
          const int s = X.src[qy * 2 + qx];
          const T* av = buf_of(OLD, HO.plevel[s], 0);
          const int li = fi - qx * m, lj = fj - qy * m;
          val = 0.25 * ((double(av[at(OLD, q, s, li, lj)]) + double(av[at(OLD, q, s, li + 1, lj)])) +
                        (double(av[at(OLD, q, s, li, lj + 1)]) + double(av[at(OLD, q, s, li + 1, lj + 1)])));
        } else {
          int FX = 2 * i, FY = 2 * j;
          if (kind == 2) FY += 1;
          if (kind == 3) FX += 1;
          const int qx = min(FX / m, 1), qy = min(FY / m, 1);
          const int s = X.src[qy * 2 + qx];
          val = buf_of(OLD, HO.plevel[s], 1)[at(OLD, q, s, FX - qx * m, FY - qy * m)];
        }
      }
      NEW.p[0][kind][at(NEW, q, p, i, j)] = T(val);
    }
  }
}

// ---------------------------------------------------------------------------
// FP64 sums (global conservation): per-leaf partials, then one block.
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(kThreads) void k_sum_partial(Bufs<T> B, HierDev H, double area0, double* part) {
  const int p = blockIdx.x;
  const int l = H.plevel[p];
  const int m = B.m, nc = B.ncomp;
  const T* av = buf_of(B, l, 0);
  __shared__ double red[kThreads];
  for (int q = 0; q < nc; ++q) {
    double s = 0.0;
    for (int e = threadIdx.x; e < m * m; e += kThreads) s += double(av[at(B, q, p, e % m, e / m)]);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[size_t(p) * nc + q] = red[0] * area0 / double(1LL << (2 * l));
    __syncthreads();
  }
}

__global__ __launch_bounds__(kThreads) void k_sum_final(const double* part, int n, int nc, double* out) {
  __shared__ double red[kThreads];
  for (int q = 0; q < nc; ++q) {
    double s = 0.0;
    for (int p = threadIdx.x; p < n; p += kThreads) s += part[size_t(p) * nc + q];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[q] = red[0];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Statically allocated scratch of the allocation-free reduction
// (af_reduce_sum_noalloc): the per-leaf partial sums, kScratchSums doubles.
// Each device holds its own copy until the process ends; its device address
// is looked up once per device (hipGetSymbolAddress) and used from then on.
// Host code never passes the array's name to a kernel: on the host it is a
// stand-in, not a device address.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[kScratchSums];

hipError_t scratch_sums(double** ptr) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static double* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[dev] = static_cast<double*>(p);
  }
  *ptr = addr[dev];
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

// The weights a patch step of equation EQ takes from the host's table
// (acoustics: the orbit form of AcAllWeights).
template <typename T, int EQ>
static const typename WSel<T, EQ>::type& step_weights(const void* p) {
  if constexpr (EQ == 1)
    return static_cast<const AcAllWeights<T>*>(p)->orbit;
  else
    return *static_cast<const typename WSel<T, EQ>::type*>(p);
}

template <typename T, int EQ, int M, int TY>
static hipError_t launch_step_t(const StepLaunch& s, hipStream_t st) {
  StepArgs<T> A;
  for (int k = 0; k < 4; ++k) {
    A.in[k] = static_cast<const T*>(s.in[k]);
    A.out[k] = static_cast<T*>(s.out[k]);
  }
  A.npatch = s.npatch; A.pitch = s.pitch; A.first = s.first; A.region = s.region;
  A.dtdx = T(s.dtdx); A.dtdy = T(s.dtdy);
  A.a = T(s.a); A.b = T(s.b); A.c = T(s.c);
  A.len_dt_x = s.len_dt_x; A.len_dt_y = s.len_dt_y;
  A.reg = s.reg; A.side_mask = s.side_mask; A.leaf_xy = s.leaf_xy; A.gnx = s.gnx; A.gny = s.gny;
  const int span = M + 2 * s.region;
  const int tiles = (span + TY - 1) / TY;
  const dim3 grid(unsigned(s.count * tiles));
  const auto& W = step_weights<T, EQ>(s.weights);
  if (s.gnx > 0)
    hipLaunchKernelGGL((k_patch_step<T, EQ, M, TY, true>), grid, dim3(kThreads), 0, st, A, W);
  else
    hipLaunchKernelGGL((k_patch_step<T, EQ, M, TY, false>), grid, dim3(kThreads), 0, st, A, W);
  return hipGetLastError();
}

template <typename T, int EQ>
static hipError_t launch_step_m(const StepLaunch& s, hipStream_t st) {
  // tile heights chosen so that a tile holds about 256 cells
  switch (s.m) {
    case 8: return launch_step_t<T, EQ, 8, 8>(s, st);
    case 16: return s.ty == 8 ? launch_step_t<T, EQ, 16, 8>(s, st) : launch_step_t<T, EQ, 16, 16>(s, st);
    case 32: return s.ty == 4 ? launch_step_t<T, EQ, 32, 4>(s, st) : launch_step_t<T, EQ, 32, 8>(s, st);
    case 64: return s.ty == 2 ? launch_step_t<T, EQ, 64, 2>(s, st) : launch_step_t<T, EQ, 64, 4>(s, st);
    case 128: return launch_step_t<T, EQ, 128, 2>(s, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_patch_step(const StepLaunch& s, hipStream_t st) {
  if (s.count <= 0) return hipSuccess;
  switch (s.eq) {
    case 0: return s.fp32 ? launch_step_m<float, 0>(s, st) : launch_step_m<double, 0>(s, st);
    case 1: return s.fp32 ? launch_step_m<float, 1>(s, st) : launch_step_m<double, 1>(s, st);
    case 2: return s.fp32 ? launch_step_m<float, 2>(s, st) : launch_step_m<double, 2>(s, st);
    case 3: return s.fp32 ? launch_step_m<float, 3>(s, st) : launch_step_m<double, 3>(s, st);
    case 4: return s.fp32 ? launch_step_m<float, 4>(s, st) : launch_step_m<double, 4>(s, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int EQ, int M, int TY, bool PAIR = false>
static hipError_t launch_amr_t(const AmrStepLaunch& s, hipStream_t st) {
  AmrStepArgs<T> A;
  for (int b = 0; b < 2; ++b)
    for (int k = 0; k < 4; ++k) A.p[b][k] = static_cast<T*>(s.p[b][k]);
  A.npatch = s.npatch;
  A.pitch = s.pitch;
  A.mask = s.mask;
  A.nlev = s.nlev;
  A.lev0 = s.lev0;
  int blocks = 0;
  for (int k = 0; k < s.nlev; ++k) {
    const int span = M + 2 * s.region[k];
    const int tiles = (span + TY - 1) / TY;
    A.first[k] = s.first[k];
    A.region[k] = s.region[k];
    A.tiles[k] = tiles;
    A.rows[k] = (span + tiles - 1) / tiles;
    A.len_dt_x[k] = s.len_dt_x[k];
    A.len_dt_y[k] = s.len_dt_y[k];
    A.items[k] = s.count[k] * tiles;
  }
  for (int kk = 0; kk < s.nlev; ++kk) {
    A.bstart[kk] = blocks;
    blocks += (A.items[s.nlev - 1 - kk] + 7) / 8 * 8;
  }
  A.bstart[s.nlev] = blocks;
  if (blocks == 0) return hipSuccess;
  A.dtdx = T(s.dtdx); A.dtdy = T(s.dtdy);
  A.a = T(s.a); A.b = T(s.b); A.c = T(s.c);
  A.reg = s.reg;
  A.side_mask = s.side_mask;
  A.plan = s.plan;
  A.entries = s.entries;
  A.nentries = s.nentries;
  A.ninner = s.ninner;
  A.fw = s.fw;
  A.nbr = s.nbr;
  A.gnflags = s.gnflags;
  A.pair = PAIR && s.pair;
  const auto* wdev = static_cast<const AcOrbitWeights<T>*>(s.weights_dev);
  const auto& W = step_weights<T, EQ>(s.weights);
  hipLaunchKernelGGL((k_amr_step<T, EQ, M, TY, PAIR>), dim3(unsigned(blocks)), dim3(kThreads), 0, st, A, W, wdev);
  return hipGetLastError();
}

template <typename T, int EQ>
static hipError_t launch_amr_m(const AmrStepLaunch& s, hipStream_t st) {
  if (s.pair) {
    switch (s.m) {
      case 8: return launch_amr_t<T, EQ, 8, 10, true>(s, st);
      case 16: return launch_amr_t<T, EQ, 16, 18, true>(s, st);
      default: return hipErrorInvalidValue;
    }
  }
  switch (s.m) {
    case 8: return launch_amr_t<T, EQ, 8, 8>(s, st);
    case 16: return s.ty == 8 ? launch_amr_t<T, EQ, 16, 8>(s, st) : launch_amr_t<T, EQ, 16, 16>(s, st);
    case 32: return s.ty == 4 ? launch_amr_t<T, EQ, 32, 4>(s, st) : launch_amr_t<T, EQ, 32, 8>(s, st);
    case 64: return s.ty == 2 ? launch_amr_t<T, EQ, 64, 2>(s, st) : launch_amr_t<T, EQ, 64, 4>(s, st);
    case 128: return launch_amr_t<T, EQ, 128, 2>(s, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_amr_step(const AmrStepLaunch& s, hipStream_t st) {
  if (s.nlev <= 0) return hipSuccess;
  switch (s.eq) {
    case 0: return s.fp32 ? launch_amr_m<float, 0>(s, st) : launch_amr_m<double, 0>(s, st);
    case 1: return s.fp32 ? launch_amr_m<float, 1>(s, st) : launch_amr_m<double, 1>(s, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
static Bufs<T> make_bufs(const BufLaunch& b);

template <typename T>
static hipError_t launch_sync_t(const AmrSyncLaunch& s, hipStream_t st) {
  AmrSyncArgs<T> A;
  A.B = make_bufs<T>(s.b);
  A.plevel = s.plevel;
  A.cops = s.cops;
  A.ncops = s.ncops;
  A.faces = s.faces;
  A.nfaces = s.nfaces;
  A.reg = s.reg;
  A.inv_area0 = s.inv_area0;
  const int blocks = (s.ncops + kThreads - 1) / kThreads + (s.nfaces + kThreads - 1) / kThreads;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_amr_sync<T>, dim3(unsigned(blocks)), dim3(kThreads), 0, st, A);
  return hipGetLastError();
}

hipError_t launch_amr_sync(const AmrSyncLaunch& s, hipStream_t st) {
  return s.fp32 ? launch_sync_t<float>(s, st) : launch_sync_t<double>(s, st);
}

hipError_t launch_canon_ops(const int4* plan, const int32_t* entries, int nentries, const int32_t* bnd, int nbnd,
                            const int32_t* canon, int ncanon, const int32_t* plevel, int4* ops, hipStream_t st) {
  const long n = long(ncanon) * nbnd;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_canon_ops, dim3(unsigned(std::min<long>((n + kThreads - 1) / kThreads, 4096))),
                     dim3(kThreads), 0, st, plan, entries, nentries, bnd, nbnd, canon, ncanon, plevel, ops);
  return hipGetLastError();
}

bool step_shape_supported(int m, int ty) {
  switch (m) {
    case 8: return ty == 8;
    case 16: return ty == 8 || ty == 16;
    case 32: return ty == 4 || ty == 8;
    case 64: return ty == 2 || ty == 4;
    case 128: return ty == 2;
    default: return false;
  }
}

template <typename T>
static AdvanceArgs<T> advance_args(const AdvanceLaunch& s) {
  AdvanceArgs<T> A;
  for (int k = 0; k < 4; ++k) {
    A.in[k] = static_cast<const T*>(s.in[k]);
    A.out[k] = static_cast<T*>(s.out[k]);
  }
  A.npatch = s.npatch; A.pitch = s.pitch; A.first = s.first; A.nx = s.nx; A.ny = s.ny;
  A.dtdx = T(s.dtdx); A.dtdy = T(s.dtdy); A.a = T(s.a); A.b = T(s.b); A.c = T(s.c);
  return A;
}

// Whether every node kind takes its source cells in the upwind pattern.
template <typename T>
static bool adv_up_pattern(const AdvWeights<T>& W) {
  bool up = true;
  for (int k = 0; k < 3; ++k)
    for (int t = 0; t < 2; ++t) up = up && W.off[k][t][0] == up_off(k, 0) && W.off[k][t][1] == up_off(k, 1);
  return up;
}

bool level_advance_up_pattern(bool fp32, int eq, const void* weights) {
  if (eq != 0) return false;
  return fp32 ? adv_up_pattern(*static_cast<const AdvWeights<float>*>(weights))
              : adv_up_pattern(*static_cast<const AdvWeights<double>*>(weights));
}

template <typename T, int EQ, int M, int K, int NT>
static hipError_t launch_adv_t(const AdvanceLaunch& s, hipStream_t st) {
  const AdvanceArgs<T> A = advance_args<T>(s);
  const dim3 grid(unsigned(s.count));
  if constexpr (EQ == 0) {
    const AdvWeights<T>& W = *static_cast<const AdvWeights<T>*>(s.weights);
    bool ss = true;
    for (int k = 0; k < 3; ++k)
      for (int t = 0; t < 2; ++t) ss = ss && W.off[k][t][0] == W.off[k][0][0] && W.off[k][t][1] == W.off[k][0][1];
    if (adv_up_pattern(W))
      hipLaunchKernelGGL((k_level_advance_up<T, M, K, NT>), grid, dim3(NT), 0, st, A, W);
    else if (ss)
      hipLaunchKernelGGL((k_level_advance_adv<T, M, K, NT, true>), grid, dim3(NT), 0, st, A, W);
    else
      hipLaunchKernelGGL((k_level_advance_adv<T, M, K, NT, false>), grid, dim3(NT), 0, st, A, W);
  } else {
    hipLaunchKernelGGL((k_level_advance<T, M, K, NT>), grid, dim3(NT), 0, st, A,
                       static_cast<const AcAllWeights<T>*>(s.weights)->dense);
  }
  return hipGetLastError();
}

// Supported (m, K, threads) shapes of the level advance, per precision and
// equation.  LDS: advection 10 E^2 words, acoustics 21 E^2 words, with
// E = m + 2K + 1.
#define AF_ADV_SHAPES(X)                                                                                 \
  X(float, 0, 32, 1, 256) X(float, 0, 32, 2, 256) X(float, 0, 32, 2, 512) X(float, 0, 32, 4, 512)      \
  X(float, 0, 32, 4, 1024) X(float, 0, 32, 5, 1024) X(float, 0, 32, 6, 768) X(float, 0, 32, 6, 1024)   \
  X(float, 0, 32, 7, 1024) X(float, 0, 32, 8, 512) X(float, 0, 32, 8, 1024) X(float, 0, 32, 5, 512)     \
  X(float, 0, 32, 6, 512) X(float, 0, 32, 10, 1024)                                                     \
  X(float, 0, 16, 1, 256) X(float, 0, 16, 2, 256) X(float, 0, 16, 4, 256) X(float, 0, 16, 8, 256)      \
  X(double, 0, 32, 1, 256) X(double, 0, 32, 2, 512) X(double, 0, 32, 3, 1024) X(double, 0, 32, 4, 512) \
  X(double, 0, 32, 4, 1024) X(double, 0, 32, 5, 1024)                                                   \
  X(double, 0, 16, 1, 256) X(double, 0, 16, 2, 256) X(double, 0, 16, 4, 256)                            \
  X(float, 1, 16, 1, 256) X(float, 1, 16, 2, 256) X(float, 1, 32, 1, 512) X(float, 1, 32, 2, 512)      \
  X(double, 1, 16, 1, 256) X(double, 1, 16, 2, 256)

// Advection shapes that only the upwind one-pass kernel runs: its gathered
// block has side m + K + 1, where the two-pass kernel's LDS would not hold
// m + 2K + 1.  LDS: 8 arrays of (m + K + R + 1) rows of a bank-aligned pitch.
#define AF_UP_SHAPES(X)                                                                                  \
  X(float, 32, 12, 1024) X(float, 32, 14, 1024) X(float, 32, 16, 1024) X(float, 32, 18, 1024)            \
  X(float, 32, 20, 1024) X(float, 32, 10, 512)                                                          \
  X(float, 32, 12, 512) X(float, 16, 12, 256) X(float, 16, 16, 256)                                      \
  X(double, 32, 6, 1024) X(double, 32, 8, 1024) X(double, 32, 10, 1024) X(double, 32, 12, 1024)           \
  X(double, 16, 8, 256)

template <typename T, int M, int K, int NT>
static hipError_t launch_up_t(const AdvanceLaunch& s, hipStream_t st) {
  const AdvWeights<T>& W = *static_cast<const AdvWeights<T>*>(s.weights);
  if (!adv_up_pattern(W)) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_level_advance_up<T, M, K, NT>), dim3(unsigned(s.count)), dim3(NT), 0, st, advance_args<T>(s),
                     W);
  return hipGetLastError();
}

hipError_t launch_level_advance(const AdvanceLaunch& s, hipStream_t st) {
  if (s.count <= 0) return hipSuccess;
#define AF_ADV_CASE(T_, EQ_, M_, K_, NT_)                                                                  \
  if ((std::is_same<T_, float>::value == s.fp32) && s.eq == EQ_ && s.m == M_ && s.k == K_ && s.nt == NT_) \
    return launch_adv_t<T_, EQ_, M_, K_, NT_>(s, st);
  AF_ADV_SHAPES(AF_ADV_CASE)
#undef AF_ADV_CASE
#define AF_UP_CASE(T_, M_, K_, NT_)                                                                      \
  if ((std::is_same<T_, float>::value == s.fp32) && s.eq == 0 && s.m == M_ && s.k == K_ && s.nt == NT_) \
    return launch_up_t<T_, M_, K_, NT_>(s, st);
  AF_UP_SHAPES(AF_UP_CASE)
#undef AF_UP_CASE
  return hipErrorInvalidValue;
}

int level_advance_shapes(bool fp32, int eq, int m, int* ks, int* nts, int cap, bool up) {
  int n = 0;
#define AF_ADV_LIST(T_, EQ_, M_, K_, NT_)                                                  \
  if ((std::is_same<T_, float>::value == fp32) && eq == EQ_ && m == M_ && n < cap) { \
    ks[n] = K_;                                                                           \
    nts[n] = NT_;                                                                         \
    ++n;                                                                                  \
  }
  AF_ADV_SHAPES(AF_ADV_LIST)
#undef AF_ADV_LIST
#define AF_UP_LIST(T_, M_, K_, NT_)                                                                \
  if (up && (std::is_same<T_, float>::value == fp32) && eq == 0 && m == M_ && n < cap) { \
    ks[n] = K_;                                                                                   \
    nts[n] = NT_;                                                                                 \
    ++n;                                                                                          \
  }
  AF_UP_SHAPES(AF_UP_LIST)
#undef AF_UP_LIST
  return n;
}

template <typename T>
static Bufs<T> make_bufs(const BufLaunch& b) {
  Bufs<T> B;
  for (int s = 0; s < 2; ++s)
    for (int k = 0; k < 4; ++k) B.p[s][k] = static_cast<T*>(b.p[s][k]);
  B.npatch = b.npatch; B.pitch = b.pitch; B.m = b.m; B.ncomp = b.ncomp; B.mask = b.mask;
  return B;
}

// Vector FMA rate probe: every thread runs 8 independent FMA chains of
// `iters` steps (enough chains to cover the FMA latency) and writes their sum,
// so nothing is dead.  Compiled with the same flags as the kernels above
// (packed FP32 off), it measures the vector rate those kernels can reach.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_fma_probe(T* out, int iters, T a, T b) {
  T x[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = T(threadIdx.x + k);
#pragma unroll 1
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int r = 0; r < 16; ++r)
#pragma unroll
      for (int k = 0; k < 8; ++k) x[k] = x[k] * a + b;
  }
  T s = T(0);
#pragma unroll
  for (int k = 0; k < 8; ++k) s += x[k];
  out[size_t(blockIdx.x) * kThreads + threadIdx.x] = s;
}

hipError_t launch_fma_probe(bool fp32, void* out, int nblocks, int iters, hipStream_t st) {
  if (fp32)
    hipLaunchKernelGGL(k_fma_probe<float>, dim3(unsigned(nblocks)), dim3(kThreads), 0, st, static_cast<float*>(out),
                       iters, 0.999999f, 1e-7f);
  else
    hipLaunchKernelGGL(k_fma_probe<double>, dim3(unsigned(nblocks)), dim3(kThreads), 0, st,
                       static_cast<double*>(out), iters, 0.999999, 1e-7);
  return hipGetLastError();
}

hipError_t launch_fill_plan(const HierDev& H, const int32_t* entries, int nentries, int m, int smin, int4* plan,
                            uint32_t* flags, int32_t* nbr, uint32_t* gnflags, hipStream_t st) {
  if (H.nleaves <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_plan, dim3(unsigned(H.nleaves)), dim3(kThreads), 0, st, H, entries, nentries, m, smin, plan,
                     flags, nbr, gnflags);
  return hipGetLastError();
}

template <typename T>
static hipError_t fill_apply_t(const BufLaunch& b, const HierDev& H, const int32_t* entries, int nentries,
                               const int4* plan, const uint32_t* flags, const FillWeights* W, int first_target,
                               int ntargets, int phase, hipStream_t st) {
  FillArgs<T> A;
  A.B = make_bufs<T>(b);
  A.plevel = H.plevel;
  A.entries = entries;
  A.plan = plan;
  A.flags = flags;
  A.W = W;
  A.nentries = nentries;
  A.chunks = (nentries + kThreads - 1) / kThreads;
  A.first_target = first_target;
  A.phase = phase;
  hipLaunchKernelGGL(k_fill_apply<T>, dim3(unsigned(ntargets * A.chunks)), dim3(kThreads), 0, st, A);
  return hipGetLastError();
}

hipError_t launch_fill_apply(bool fp32, const BufLaunch& b, const HierDev& H, const int32_t* entries, int nentries,
                             const int4* plan, const uint32_t* flags, const FillWeights* W, int first_target,
                             int ntargets, int phase, hipStream_t st) {
  if (ntargets <= 0) return hipSuccess;
  return fp32 ? fill_apply_t<float>(b, H, entries, nentries, plan, flags, W, first_target, ntargets, phase, st)
              : fill_apply_t<double>(b, H, entries, nentries, plan, flags, W, first_target, ntargets, phase, st);
}

hipError_t launch_flux_correct(bool fp32, const BufLaunch& b, const CFFace* faces, int nfaces, double* reg,
                               int level, double inv_area, hipStream_t st) {
  if (nfaces <= 0) return hipSuccess;
  const dim3 grid(unsigned((nfaces + kThreads - 1) / kThreads));
  if (fp32)
    hipLaunchKernelGGL(k_flux_correct<float>, grid, dim3(kThreads), 0, st, make_bufs<float>(b), faces, nfaces,
                       reg, level, inv_area);
  else
    hipLaunchKernelGGL(k_flux_correct<double>, grid, dim3(kThreads), 0, st, make_bufs<double>(b), faces, nfaces,
                       reg, level, inv_area);
  return hipGetLastError();
}

hipError_t launch_tag(bool fp32, const BufLaunch& b, const HierDev& H, int mode, int comp, double inv2dx0,
                      double inv2dy0, double tr, double tc, int8_t* tags, double* values, hipStream_t st) {
  if (H.nleaves <= 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL(k_tag<float>, dim3(unsigned(H.nleaves)), dim3(kThreads), 0, st, make_bufs<float>(b), H,
                       mode, comp, inv2dx0, inv2dy0, tr, tc, tags, values);
  else
    hipLaunchKernelGGL(k_tag<double>, dim3(unsigned(H.nleaves)), dim3(kThreads), 0, st, make_bufs<double>(b), H,
                       mode, comp, inv2dx0, inv2dy0, tr, tc, tags, values);
  return hipGetLastError();
}

hipError_t launch_transfer(bool fp32, const BufLaunch& old_b, const HierDev& HO, const BufLaunch& new_b,
                           const Transfer* tr, int nnew, hipStream_t st) {
  if (nnew <= 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL(k_transfer<float>, dim3(unsigned(nnew)), dim3(kThreads), 0, st, make_bufs<float>(old_b),
                       HO, make_bufs<float>(new_b), tr);
  else
    hipLaunchKernelGGL(k_transfer<double>, dim3(unsigned(nnew)), dim3(kThreads), 0, st, make_bufs<double>(old_b),
                       HO, make_bufs<double>(new_b), tr);
  return hipGetLastError();
}

hipError_t launch_sum(bool fp32, const BufLaunch& b, const HierDev& H, double area0, double* part, double* out,
                      hipStream_t st) {
  if (H.nleaves <= 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL(k_sum_partial<float>, dim3(unsigned(H.nleaves)), dim3(kThreads), 0, st,
                       make_bufs<float>(b), H, area0, part);
  else
    hipLaunchKernelGGL(k_sum_partial<double>, dim3(unsigned(H.nleaves)), dim3(kThreads), 0, st,
                       make_bufs<double>(b), H, area0, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kThreads), 0, st, part, H.nleaves, b.ncomp, out);
  return hipGetLastError();
}

}  // namespace af
