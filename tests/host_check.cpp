// Host precompute of the library (paper_2602_16591_amd/csrc/host.cpp) driven on its own, for a
// build under the address and undefined-behaviour sanitizers (test infrastructure: compiled
// and run by tests/test_host_sanitizers.py). Runs Alg. 3 (cube and cuboid), the PSWF solve of
// App. B, the scaling and window tables, the residual table, the oversampled grid and the
// twiddle tables, and prints one JSON object per line, which the test compares with what the
// optimised library returns for the same arguments.
#include <cmath>
#include <cstdio>
#include <vector>

#include "host.hpp"

namespace {

// the window fit tolerance the library uses for a float32 (f32 != 0) or float64 plan
double fit_tol(double eps, int f32) { return std::fmax(0.01 * eps, f32 ? 5e-9 : 1e-15); }

void print_list(const char* key, const std::vector<double>& v) {
  std::printf(", \"%s\": [", key);
  for (size_t i = 0; i < v.size(); ++i) std::printf("%s%.17g", i ? ", " : "", v[i]);
  std::printf("]");
}

void print_params(const pswfe::Params& p) {
  std::printf("\"m\": %d, \"my\": %d, \"mz\": %d, \"P\": %d, \"rc\": %.17g, \"cs\": %.17g, \"cw\": %.17g, "
              "\"alpha\": %.17g",
              p.m, p.grid(1), p.grid(2), p.P, p.rc, p.cs, p.cw, p.alpha);
}

struct Case {
  const char* name;
  double eps, L, rc;
  int m;
  long long n;
  double q_l2;
  int tol_mode, f32;
};

}  // namespace

int main() {
  const Case cases[] = {
      {"rel_m64", 1e-6, 1.0, 0.0, 64, 0, 0.0, 0, 1},
      {"rel_m30_L1.3", 1e-4, 1.3, 0.0, 30, 0, 0.0, 0, 1},
      {"rel_rc_eps1e-10", 1e-10, 1.0, 0.15, 0, 0, 0.0, 0, 0},
      {"abs_rc", 1e-6, 1.0, 0.15, 0, 0, 10.0, 1, 1},
      {"rel_n5000_L1.5", 1e-6, 1.5, 0.0, 0, 5000, 0.0, 0, 1},
  };
  int bad = 0;
  for (const Case& c : cases) {
    pswfe::Params p{};
    const int st = pswfe::choose_params(c.eps, c.L, c.rc, c.m, c.n, c.q_l2, c.tol_mode, &p);
    std::printf("{\"case\": \"%s\", \"status\": %d, ", c.name, st);
    if (st != 0) {
      std::printf("\"m\": 0}\n");
      ++bad;
      continue;
    }
    print_params(p);
    pswfe::Tables t;
    pswfe::build_tables(p, 0, fit_tol(c.eps, c.f32), &t);
    std::printf(", \"deg\": %d, \"fit_err\": %.17g, \"self_coef\": %.17g", t.deg, t.fit_err, t.self_coef);
    print_list("coef", t.coef);
    print_list("w", t.w);
    print_list("tm", t.tm);
    pswfe::LocalTable lt;
    pswfe::build_local_table(p, c.f32 ? 1e-10 : 1e-15, &lt);
    std::printf(", \"local_deg\": %d, \"local_K\": %.17g", lt.deg, lt.K);
    pswfe::Params q{};
    const int so = pswfe::oversample_params(p, 1.5, &q);
    std::printf(", \"over_status\": %d, \"over_m\": %d, \"over_P\": %d}\n", so, q.m, q.P);
  }
  {
    pswfe::Params p{};
    const int st = pswfe::choose_params_box(1e-6, 1.0, 1.3, 0.8, 0.15, 0, 0, 0.0, 0, &p);
    std::printf("{\"case\": \"box\", \"status\": %d, ", st);
    print_params(p);
    pswfe::Tables t;
    if (st == 0) pswfe::build_tables(p, 0, fit_tol(1e-6, 1), &t);
    std::printf(", \"deg\": %d", t.deg);
    print_list("coef", t.coef);
    std::printf("}\n");
    if (st != 0) ++bad;
  }
  {
    std::vector<double> tw;
    pswfe::twiddles(60, 1, &tw);
    const pswfe::Pswf f(20.0);
    std::printf("{\"case\": \"misc\", \"tw_len\": %zu, \"tw_7\": [%.17g, %.17g], \"w0_1\": %.17g, \"wm1\": %.17g, "
                "\"chi0_20\": %.17g, \"lambda0_20\": %.17g, \"psi_0.3\": %.17g}\n",
                tw.size(), tw[14], tw[15], pswfe::lambert_w0(1.0), pswfe::lambert_wm1(-0.2), f.chi0, f.lambda0,
                f.psi(0.3));
  }
  return bad;
}
