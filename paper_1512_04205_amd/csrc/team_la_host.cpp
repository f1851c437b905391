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
  std::vector<double> T((size_t)Jmax + k + 6 * (size_t)Jmax * k);
  std::vector<double> Q((size_t)(Jmax + 1) * N), V((size_t)N * k), TV((size_t)N * k), At(k * k), Hs(k * k);
  std::vector<cpx> LU((size_t)k * k * k), bb((size_t)k * k), yy((size_t)k * k);
  std::vector<int> piv((size_t)k * k), flag(1);
  SmallLAWork ws;
  const int64_t fastd = 15488;  // as the device's LDS region
  std::vector<double> fast(fastd);
  ws.lz = LanczosWork{q.data(), w.data(), h.data(), alpha.data(), beta.data(), T.data(),
                      fast.data(), fastd};
  ws.Q = Q.data();
  ws.V = V.data();
  ws.TV = TV.data();
  ws.At = At.data();
  ws.Hs = Hs.data();
  ws.LU = LU.data();
  ws.bb = bb.data();
  ws.yy = yy.data();
  ws.piv = piv.data();
  ws.flag = flag.data();
  HostTeam tm;
  return small_la_run(tm, Gr, m, k, rtol, Jmax, scale, ws, mu, sigma, reinterpret_cast<cpx*>(lam),
                      reinterpret_cast<cpx*>(W), reinterpret_cast<cpx*>(G), J);
}

}  // namespace cdmd
