// opcount.cpp -- algorithmic operation count of the device arithmetic of one
// 2D interface (prologue, hydrodynamic part, the two kinetic parts) and one
// cell (reconstruction of the four conservative variables with its
// admissibility test), by running the device functions of gks_device.h and
// interface_gen.h on the host with counting scalar types (count_scalar.h):
// double -> D, the compute type -> F (FP32-mixed form) or D (FP64 form).
// Built and run by opcount.py, which writes opcounts.json.  The few
// operations that gks.hip itself adds (the accumulation of each phase into
// the stored flux and point values, the Prandtl-number fix, the update) are
// listed in opcount.py.
#include <cmath>
#include <cstdio>
#include <cstring>

#include "count_scalar.h"

using gks_opcount::D;
using gks_opcount::F;
using gks_opcount::counts;
using gks_opcount::erfc;
using gks_opcount::exp;
using gks_opcount::sqrt;

#define double ::gks_opcount::D
#include "gks_device.h"
#undef double

namespace {

// a smooth state around the interface: averages, reconstruction
// coefficients and the six averages of the equilibrium stencil (values of
// an isentropic-vortex-like field); viscous selects the Navier-Stokes terms
template <typename TC>
void one_interface(bool viscous, long long (&out)[3]) {
  using namespace gks;
  Phys P;
  std::memset((void*)&P, 0, sizeof(P));
  P.gamma = 1.4;
  P.K = (4.0 - 2.0 * 1.4) / 0.4;
  P.nth = 5.0;
  P.kp[0] = 1.0;
  for (int e = 1; e < 4; ++e) P.kp[e] = P.kp[e - 1] * (P.K + 2.0 * (e - 1));
  P.tau_eps = 0.05;
  P.tau_c = 1.0;
  P.mu = viscous ? 1e-3 : 0.0;
  P.prfix = viscous ? 1.0 / 0.72 - 1.0 : 0.0;
  P.viscous = viscous ? 1 : 0;
  const D dt = 2.5e-3, hn = 0.04, hs = 0.04;
  D Wc[2][4], pc[2][4][5], Ueq[2][3][4];
  for (int s = 0; s < 2; ++s)
    for (int v = 0; v < 4; ++v) {
      const double base[4] = {1.0, 0.9, 1.1, 3.3};
      Wc[s][v] = base[v] * (1.0 + 0.01 * s);
      for (int m = 0; m < 5; ++m) pc[s][v][m] = 0.05 * (1 + m) * (v + 1) * (s ? -1.0 : 1.0);
    }
  for (int m = 0; m < 2; ++m)
    for (int n = 0; n < 3; ++n)
      for (int v = 0; v < 4; ++v) Ueq[m][n][v] = Wc[m][v] * (1.0 + 0.002 * (n - 1));
  D recd[ND_REC];
  TC rect[nt_rec<TC>()];
  Rec<TC> R{recd, rect, 1};
  D flux[4], pv[4], pvm[4], pvp[4], E[4];
  counts() = gks_opcount::Counts();
  if (!iface_prologue_2d<TC>(P, dt, hn, hs, Wc, pc, Ueq, R, 0, flux, pv)) std::fprintf(stderr, "nonphysical\n");
  iface_hydro_2d<TC>(P, dt, hs, R, 0, flux, pvm, pvp, E);
  for (int s = 0; s < 2; ++s) iface_kinetic_2d<TC>(P, dt, hn, hs, s, Wc[s], pc[s], R, 0, flux, pvm, pvp, E);
  out[0] = counts().d;
  out[1] = counts().f;
  out[2] = counts().dtrans;
}

void one_cell(long long (&out)[3]) {
  using namespace gks;
  const double h = 0.04, k = 0.04;
  D S[13][4], p[4][5], Wc[4];
  for (int q = 0; q < 13; ++q)
    for (int v = 0; v < 4; ++v) {
      const double base[4] = {1.0, 0.9, 1.1, 3.3};
      S[q][v] = base[v] * (1.0 + 0.003 * q * (v + 1) - 0.0004 * q * q);
    }
  counts() = gks_opcount::Counts();
  const ReconDiv Dv(h, k);
  for (int v = 0; v < 4; ++v) {
    Wc[v] = S[0][v];
    recon_2d(S[0][v], S[1][v], S[2][v], S[3][v], S[4][v], S[5][v], S[6][v], S[7][v], S[8][v], S[9][v], S[10][v],
             S[11][v], S[12][v], h, k, 1e-6, 10.0, Dv, 1.4210854715202004e-14, p[v]);
  }
  Range rg;
  for (int q = 0; q < 5; ++q) rg.add(S[q][0], pressure_2d(1.4, S[q]));
  (void)recon_admissible_2d(Wc, p, h, k, 1.4, rg, 1);
  out[0] = counts().d;
  out[1] = counts().f;
  out[2] = counts().dtrans;
}

}  // namespace

int main() {
  long long a[3], b[3], c[3], d[3], e[3];
  one_interface<F>(false, a);
  one_interface<F>(true, b);
  one_interface<D>(false, c);
  one_interface<D>(true, d);
  one_cell(e);
  std::printf("{\"interface_euler_fp32_mixed\": [%lld, %lld, %lld], \"interface_ns_fp32_mixed\": [%lld, %lld, %lld], "
              "\"interface_euler_fp64\": [%lld, %lld, %lld], \"interface_ns_fp64\": [%lld, %lld, %lld], "
              "\"recon_cell\": [%lld, %lld, %lld]}\n",
              a[0], a[1], a[2], b[0], b[1], b[2], c[0], c[1], c[2], d[0], d[1], d[2], e[0], e[1], e[2]);
  return 0;
}
