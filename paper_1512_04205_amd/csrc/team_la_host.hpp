// Host run of the team small linear algebra; see team_la.hpp.
#pragma once

namespace cdmd {
// groups: 1 = one thread; more = the Lanczos rows split over that many host threads.
// lam: 2k (re, im); W: 2k*k (column j at 2*j*k); G: 2N*k (row t at 2*t*k).
int team_small_la_host(const double* Gr, int m, int k, double rtol, int Jmax, double scale, int groups,
                       double* mu, double* sigma, double* lam, double* W, double* G, int* J);
}
