// Driver for the sanitizer build of the library's host-only code
// (csrc/host_constants.cpp, csrc/quadrature_search.cpp), compiled with g++
// and -fsanitize=address,undefined by tests/test_sanitizers.py.  It runs
// every host entry point of that code once -- the polished quadrature and
// force matrices with their self-checks, the Maxwell-Juttner moments, the
// massive and massless quadrature searches, their error paths -- and prints
// the results, one "key value..." line each.
//
// Usage: host_driver mbar x0 y0 x1 y1 ...   (the massive search's vectors)
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../include/rlbm_quadrature.h"
#include "../../paper_1804_02418_amd/csrc/rlbm_internal.h"

namespace rlbm {
// The library defines this in its lattice runtime, which is not built here.
rlbm_status set_error(rlbm_status st, const char *msg)
{
    if (msg && std::getenv("HOST_DRIVER_VERBOSE")) std::fprintf(stderr, "error: %s\n", msg);
    return st;
}
}  // namespace rlbm

int main(int argc, char **argv)
{
    if (argc < 4 || (argc - 2) % 2) {
        std::fprintf(stderr, "usage: %s mbar x0 y0 x1 y1 ...\n", argv[0]);
        return 2;
    }
    // polished quadrature and force matrices
    rlbm::Quadrature q;
    double Cx[rlbm::kK][rlbm::kK], Cy[rlbm::kK][rlbm::kK];
    const char *err = nullptr;
    if (!rlbm::host_constants(&q, Cx, Cy, &err)) {
        std::printf("host_constants_failed %s\n", err ? err : "?");
        return 1;
    }
    std::printf("w1 %.17g %.17g %.17g %.17g\n", q.w1[0], q.w1[1], q.w1[2], q.w1[3]);
    std::printf("w2 %.17g %.17g %.17g %.17g\n", q.w2[0], q.w2[1], q.w2[2], q.w2[3]);
    std::printf("p0 %.17g %.17g %.17g %.17g\n", q.p0[0], q.p0[1], q.p0[2], q.p0[3]);
    std::printf("Cx01 %.17g Cy03 %.17g\n", Cx[0][2], Cy[0][3]);
    std::printf("massless_residual %.17g\n", rlbm::massless_stencil_residual(q));
    // Maxwell-Juttner moments
    const int abc[][3] = {{0, 0, 0}, {1, 0, 0}, {3, 2, 0}, {0, 2, 4}, {1, 4, 2}, {2, 0, 6}};
    for (double m : {0.0, 0.5, 5.0}) {
        for (const auto &t : abc) {
            double v = 0;
            if (rlbm_mj_moment(m, t[0], t[1], t[2], &v) != RLBM_OK) return 1;
            std::printf("moment %g %d %d %d %.17g\n", m, t[0], t[1], t[2], v);
        }
    }
    // massive search on the given vectors
    const double mbar = std::atof(argv[1]);
    std::vector<int> vec;
    for (int k = 2; k < argc; ++k) vec.push_back(std::atoi(argv[k]));
    const int nvec = (int)vec.size() / 2;
    std::vector<double> w(nvec);
    double v0 = 0, wmin = 0, res = 0;
    int st = rlbm_quadrature_massive(mbar, 3, vec.data(), nvec, 2000, &v0, w.data(), &wmin, &res);
    std::printf("massive %d %.17g %.17g %.17g\n", st, v0, wmin, res);
    // massless search on the paper's 12 directions, 4 shells, from random starts
    int dirs[2 * rlbm::kDirs];
    for (int d = 0; d < rlbm::kDirs; ++d) {
        dirs[2 * d] = rlbm::kCx[d];
        dirs[2 * d + 1] = rlbm::kCy[d];
    }
    double p0[4], wl[4 * rlbm::kDirs];
    st = rlbm_quadrature_massless(3, dirs, rlbm::kDirs, 4, nullptr, nullptr, 3, 40, p0, wl, &wmin, &res);
    std::printf("massless %d %.17g %.17g %.17g %.17g %.17g %.17g\n", st, p0[0], p0[1], p0[2], p0[3], wmin, res);
    // error paths: an odd vector count, a direction of another length, a bad order
    st = rlbm_quadrature_massive(mbar, 3, vec.data(), nvec - 1, 100, &v0, w.data(), &wmin, &res);
    std::printf("massive_bad %d\n", st);
    dirs[2 * (rlbm::kDirs - 1)] = 1;
    dirs[2 * (rlbm::kDirs - 1) + 1] = 0;
    st = rlbm_quadrature_massless(3, dirs, rlbm::kDirs, 4, nullptr, nullptr, 3, 4, p0, wl, &wmin, &res);
    std::printf("massless_bad %d\n", st);
    st = rlbm_quadrature_massive(mbar, 0, vec.data(), nvec, 100, &v0, w.data(), &wmin, &res);
    std::printf("order_bad %d\n", st);
    return 0;
}
