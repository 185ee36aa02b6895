// Host-code driver for the sanitizer test (tests/test_host_sanitizers.py):
// builds trees, traversals and P2P work plans for random and degenerate
// inputs with AddressSanitizer/UndefinedBehaviorSanitizer/LeakSanitizer, and
// injects an allocation failure at every checkpoint of each build and
// traversal to check that the partial state is released.
#include <cstdio>
#include <cstdlib>
#include <new>
#include <random>
#include <string>
#include <vector>

#include "fmm_internal.h"

namespace fmmlib {
static int g_fail_at = -1, g_count = 0;
void reset_alloc_checkpoints() { g_count = 0; }
void alloc_checkpoint() {
  if (++g_count == g_fail_at) throw std::bad_alloc();
}
}  // namespace fmmlib

static int run_case(const std::vector<double> &xyz, int ncrit, double theta, bool leaf_first) {
  using namespace fmmlib;
  TreeData t;
  std::string err;
  reset_alloc_checkpoints();
  if (build_tree(xyz.data(), (int64_t)xyz.size() / 3, ncrit, t, err) != 0) return 1;
  ListData l;
  reset_alloc_checkpoints();
  dual_traverse(t, theta, leaf_first, 0, l);
  P2PPlan plan;
  if (build_p2p_plan(t, l, plan, err) != 0) return 5;
  // every body has exactly one leaf; every item covers valid ranges
  for (const auto &it : plan.items) {
    const int nt = it.tgt_cfg & 0xff;
    if (nt < 1 || nt > 64 || it.tgt_begin < 0 || it.tgt_begin + nt > t.n) return 2;
    if (it.n_runs > kP2PMaxRuns) return 3;
    if (it.out_off < 0 || it.out_off + nt > plan.n_partials) return 4;
  }
  return 0;
}

int main() {
  std::mt19937_64 rng(7);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  std::vector<std::vector<double>> inputs;
  for (int n : {0, 1, 2, 65, 3000}) {
    std::vector<double> x(3 * n);
    for (auto &v : x) v = (double)(float)U(rng);
    inputs.push_back(x);
  }
  std::vector<double> dup(3 * 500);
  for (int i = 0; i < 500; ++i)
    for (int d = 0; d < 3; ++d) dup[3 * i + d] = (i < 200) ? 0.25 : (double)(float)U(rng);
  inputs.push_back(dup);
  std::vector<double> line(3 * 400);
  for (int i = 0; i < 400; ++i) line[3 * i] = i / 399.0;
  inputs.push_back(line);
  for (const auto &x : inputs)
    for (int ncrit : {1, 8, 64})
      for (bool lf : {false, true}) {
        if (int rc = run_case(x, ncrit, 0.45, lf)) {
          std::printf("case failed rc=%d\n", rc);
          return rc;
        }
      }
  // allocation failure at each checkpoint of build / traversal
  int injected = 0;
  for (int k = 1; k <= 12; ++k) {
    fmmlib::g_fail_at = k;
    try {
      run_case(inputs[4], 8, 0.45, false);
    } catch (const std::bad_alloc &) {
      ++injected;
    }
  }
  fmmlib::g_fail_at = -1;
  std::printf("ok injected=%d\n", injected);
  return injected > 0 ? 0 : 5;
}
