// Host instantiation of the team small linear algebra, used by the cdmd_dbg_team_small_la
// test entry point and as the reference of the device solve: one thread, or Lanczos split
// over row groups run by host threads that exchange their shares through shared memory
// as the device's workgroups do through global memory.
#include <condition_variable>
#include <mutex>
#include <thread>
#include <vector>

#include "team_la.hpp"
#include "team_la_host.hpp"

namespace cdmd {
namespace {

using namespace tla;

struct HostGridShared {
  std::mutex mu;
  std::condition_variable cv;
  unsigned arrived = 0;
  int G = 1, PS = 0, N = 0, NQ = 0;
  std::vector<double> buf;  // two buffers of G*PS partials and an NQ-vector
};

// The exchange of row group g among G host threads (same contract as the device's).
struct HostGridX {
  int g = 0, G = 1, r0 = 0, r1 = 0;
  HostGridShared* sh = nullptr;
  unsigned nx = 0;
  bool exchange(HostTeam&, const double* part, int n, double* sum, const double* slice, double* full) {
    const int PS = sh->PS, N = sh->N;
    double* base = sh->buf.data() + (size_t)(nx & 1u) * ((size_t)G * PS + sh->NQ);
    for (int i = 0; i < n; ++i) base[(size_t)g * PS + i] = part[i];
    if (slice != nullptr)
      for (int t = r0; t < r1; ++t) base[(size_t)G * PS + t] = slice[t];
    ++nx;
    {
      std::unique_lock<std::mutex> lk(sh->mu);
      ++sh->arrived;
      sh->cv.notify_all();
      const unsigned target = nx * (unsigned)G;
      sh->cv.wait(lk, [&] { return sh->arrived >= target; });
    }
    for (int i = 0; i < n; ++i) {
      double v = 0.0;
      for (int q = 0; q < G; ++q) v += base[(size_t)q * PS + i];
      sum[i] = v;
    }
    if (full != nullptr)
      for (int t = 0; t < N; ++t) full[t] = base[(size_t)G * PS + t];
    return true;
  }
};

// Per-group vectors of the Lanczos work (the device's LDS arrays).
struct GroupVectors {
  std::vector<double> q, w, h, alpha, beta, fast, qc;
  GroupVectors(int N, int k, int Jmax, int64_t fastd)
      : q(N), w(N > 2 * k ? N : 2 * k), h(Jmax + 2), alpha(Jmax + 2), beta(Jmax + 2), fast(fastd),
        qc(kLaQCache) {}
};

}  // namespace

int team_small_la_host(const double* Gr, int m, int k, double rtol, int Jmax, double scale, int groups,
                       double* mu, double* sigma, double* lam, double* W, double* G, int* J) {
  const int N = m - 1;
  if (Jmax > N) Jmax = N;
  if (groups < 1) groups = 1;
  if (groups > N) groups = N;
  const SmallLALayout L = small_la_layout(N, k, Jmax);
  std::vector<double> scr((size_t)L.total);
  std::vector<int> flag(1);
  const int64_t fastd = kLaFast;  // as the device's LDS regions
  double* sp = scr.data();
  auto work = [&](GroupVectors& v) {
    SmallLAWork ws;
    ws.lz = LanczosWork{v.q.data(), v.w.data(), v.h.data(), v.alpha.data(), v.beta.data(), sp + L.T,
                        v.fast.data(), fastd, v.qc.data(), (int64_t)v.qc.size()};
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
    return ws;
  };
  std::vector<GroupVectors> gv;
  for (int g = 0; g < groups; ++g) gv.emplace_back(N, k, Jmax, fastd);
  HostTeam tm;
  if (groups == 1) {
    const SmallLAWork ws = work(gv[0]);
    return small_la_run(tm, Gr, m, k, rtol, Jmax, scale, ws, mu, sigma, reinterpret_cast<cpx*>(lam),
                        reinterpret_cast<cpx*>(W), reinterpret_cast<cpx*>(G), J);
  }
  HostGridShared sh;
  sh.G = groups;
  sh.PS = la_xps(Jmax);
  sh.N = N;
  sh.NQ = la_ldq(N);
  sh.buf.assign(2 * ((size_t)groups * sh.PS + sh.NQ), 0.0);
  std::vector<int> st(groups, 0), Js(groups, 0);
  std::vector<std::thread> th;
  for (int g = 0; g < groups; ++g)
    th.emplace_back([&, g] {
      HostTeam t;
      HostGridX xg;
      xg.g = g;
      xg.G = groups;
      la_group_rows(N, groups, g, &xg.r0, &xg.r1);
      xg.sh = &sh;
      const SmallLAWork ws = work(gv[g]);
      st[g] = small_la_phase_a(t, xg, Gr, m, k, rtol, Jmax, ws, mu, ws.Z, &Js[g]);
    });
  for (auto& t : th) t.join();
  *J = Js[0];
  // the groups agree on a failure, and otherwise on J (only group 0 tests the rank)
  const bool solved = st[0] == kOk || st[0] == kRankDeficient;
  for (int g = 1; g < groups; ++g)
    if (solved ? st[g] != kOk || Js[g] != Js[0] : st[g] != st[0]) return kDevice;
  if (st[0] != kOk) return st[0];
  const SmallLAWork ws = work(gv[0]);
  return small_la_tail(tm, Gr, m, k, *J, scale, ws, mu, sigma, reinterpret_cast<cpx*>(lam),
                       reinterpret_cast<cpx*>(W), reinterpret_cast<cpx*>(G));
}

}  // namespace cdmd
