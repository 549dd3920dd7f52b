// Host check of the library's acoustic stencils in mirror-orbit form
// (af_weights.cpp): for several Courant numbers, square and rectangular
// cells, the orbit weights exist (the dense FP64 stencils are mirror
// symmetric to 1e-12), evaluating a node orbit by orbit gives the dense
// stencil's value on random neighbourhood data, and the FP32 K weights keep
// their sums (1 for the value, 5 for the time sum) exactly.  Prints one line
// per case and exits non-zero on a failure.
#include <cmath>
#include <cstdio>
#include <random>

#include "af_internal.h"
#include "af_weights.h"

using namespace af;

int main() {
  std::mt19937_64 gen(7);
  std::normal_distribution<double> N;
  const double cases[5][2] = {{0.4, 0.4}, {0.45, 0.45}, {0.2, 0.35}, {0.5, 0.1}, {0.05, 0.05}};
  int bad = 0;
  for (const auto& cs : cases) {
    AcWeights<double> D;
    AcOrbitWeights<double> O;
    AcOrbitWeights<float> O32;
    make_ac_weights<double>(cs[0], cs[1], &D);
    const bool ok = make_ac_orbit_weights<double>(cs[0], cs[1], &O) && make_ac_orbit_weights<float>(cs[0], cs[1], &O32);
    double V[4][3][3][3];
    for (auto& a : V)
      for (auto& b : a)
        for (auto& c : b)
          for (auto& d : c) d = N(gen);
    double err = 0.0, sum_err = 0.0;
    for (int nk = 0; nk < 3; ++nk) {
      const int nb = nb_size(nk);
      // dense: value at t + dt and 4 (t + dt/2) + (t + dt)
      double dense[2][3] = {};
      for (int e = 0; e < nb; ++e) {
        const NbEntry E = nb_entry(nk, e);
        const double p = V[E.kind][0][E.dj + 1][E.di + 1], u = V[E.kind][1][E.dj + 1][E.di + 1],
                     v = V[E.kind][2][E.dj + 1][E.di + 1];
        for (int t = 0; t < 2; ++t) {
          const double* wk = nk == 0 ? D.corner[t][0] : (nk == 1 ? D.xedge[t][0] : D.yedge[t][0]);
          const double* wx = nk == 0 ? D.corner[t][1] : (nk == 1 ? D.xedge[t][1] : D.yedge[t][1]);
          const double* wy = nk == 0 ? D.corner[t][2] : (nk == 1 ? D.xedge[t][2] : D.yedge[t][2]);
          const double f = t == 0 ? 4.0 : 1.0;
          const double vp = wk[e] * p - wx[e] * u - wy[e] * v, vu = wk[e] * u - wx[e] * p, vv = wk[e] * v - wy[e] * p;
          if (t == 1) {
            dense[0][0] += vp;
            dense[0][1] += vu;
            dense[0][2] += vv;
          }
          dense[1][0] += f * vp;
          dense[1][1] += f * vu;
          dense[1][2] += f * vv;
        }
      }
      // orbit form
      for (int c = 0; c < 2; ++c) {
        double orb[3] = {};
        float ksum = 0.0f;
        double ksum_exact = 0.0;
        for (int o = 0; o < kOrbitTab[nk].n; ++o) {
          const NbOrbit& Ob = kOrbitTab[nk].o[o];
          double S[3] = {}, Dx[3] = {}, Dy[3] = {};
          for (int mb = 0; mb < Ob.n; ++mb) {
            int X = 0, Y = 0;
            nb_offset(nk, Ob.m[mb].kind, Ob.m[mb].di, Ob.m[mb].dj, &X, &Y);
            for (int q = 0; q < 3; ++q) {
              const double val = V[Ob.m[mb].kind][q][Ob.m[mb].dj + 1][Ob.m[mb].di + 1];
              S[q] += val;
              Dx[q] += (X > 0 ? 1 : (X < 0 ? -1 : 0)) * val;
              Dy[q] += (Y > 0 ? 1 : (Y < 0 ? -1 : 0)) * val;
            }
          }
          const double* w = O.w[nk][o][c];
          orb[0] += w[0] * S[0] - w[1] * Dx[1] - w[2] * Dy[2];
          orb[1] += w[0] * S[1] - w[1] * Dx[0];
          orb[2] += w[0] * S[2] - w[2] * Dy[0];
          ksum_exact += double(Ob.n) * double(O32.w[nk][o][c][0]);
          (void)ksum;
        }
        for (int q = 0; q < 3; ++q) err = std::fmax(err, std::fabs(orb[q] - dense[c][q]));
        sum_err = std::fmax(sum_err, std::fabs(ksum_exact - (c == 0 ? 1.0 : 5.0)));
      }
    }
    const bool pass = ok && err < 1e-13 && sum_err == 0.0;
    std::printf("cfl %.2f %.2f symmetric=%d max|orbit-dense|=%.3e fp32 K-sum error=%.3e %s\n", cs[0], cs[1], int(ok), err,
                sum_err, pass ? "ok" : "FAIL");
    if (!pass) ++bad;
  }
  return bad ? 1 : 0;
}
