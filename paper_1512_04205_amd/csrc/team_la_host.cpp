// Host instantiation of the team small linear algebra (one thread), used by the
// cdmd_dbg_team_small_la test entry point and as the reference of the device solve.
#include <vector>

#include "team_la.hpp"
#include "team_la_host.hpp"

namespace cdmd {

int team_small_la_host(const double* Gr, int m, int k, double rtol, int Jmax, double scale,
                       double* mu, double* sigma, double* lam, double* W, double* G, int* J) {
  using namespace tla;
  const int N = m - 1;
  if (Jmax > N) Jmax = N;
  std::vector<double> q(N), w(N > 2 * k ? N : 2 * k), h(Jmax + 2), alpha(Jmax + 2), beta(Jmax + 2);
  const SmallLALayout L = small_la_layout(N, k, Jmax);
  std::vector<double> scr((size_t)L.total);
  std::vector<int> flag(1);
  SmallLAWork ws;
  const int64_t fastd = 15488;  // as the device's LDS region
  std::vector<double> fast(fastd);
  double* sp = scr.data();
  ws.lz = LanczosWork{q.data(), w.data(), h.data(), alpha.data(), beta.data(), sp + L.T, fast.data(), fastd};
  ws.Q = sp + L.Q;
  ws.V = sp + L.V;
  ws.Z = sp + L.Z;
  ws.TV = sp + L.TV;
  ws.P = sp + L.P;
  ws.nu = sp + L.nu;
  ws.At = sp + L.At;
  ws.Hs = sp + L.Hs;
  ws.LU = reinterpret_cast<cpx*>(sp + L.LU);
  ws.bb = reinterpret_cast<cpx*>(sp + L.bb);
  ws.yy = reinterpret_cast<cpx*>(sp + L.yy);
  ws.piv = reinterpret_cast<int*>(sp + L.piv);
  ws.flag = flag.data();
  HostTeam tm;
  return small_la_run(tm, Gr, m, k, rtol, Jmax, scale, ws, mu, sigma, reinterpret_cast<cpx*>(lam),
                      reinterpret_cast<cpx*>(W), reinterpret_cast<cpx*>(G), J);
}

}  // namespace cdmd
