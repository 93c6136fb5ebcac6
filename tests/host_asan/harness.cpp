// Test infrastructure: drives the batch entry point through the CPU stand-in
// runtime (shim.cpp) in several call orders, and single problems through the
// stepping loop, and checks each report against the iteration count at which
// the stand-in stops the item.
#include <cstdio>
#include <cstdlib>
#include <vector>
#include "sgpdeconv.h"
namespace sgp { int shim_target(int b); }
struct Item { int n; float *g, *psf, *f, *f0; float b; int rank; };
int main() {
  const int sizes[4] = {16, 32, 64, 128};
  const int counts[4] = {23, 31, 17, 29};
  std::vector<Item> items;
  for (int s = 0; s < 4; ++s)
    for (int i = 0; i < counts[s]; ++i) {
      const size_t px = (size_t)sizes[s] * sizes[s];
      items.push_back(Item{sizes[s], (float*)calloc(px, 4), (float*)calloc(px, 4), (float*)calloc(px, 4),
                           (float*)calloc(px, 4), 1.f, 0});
    }
  std::vector<int> order;  // sizes interleaved, as in a generated batch
  for (int i = 0; i < (int)items.size(); ++i) order.push_back((int)((i * 37L) % items.size()));
  int bad = 0;
  auto run = [&](const std::vector<int>& idx, bool warm, int max_iter, const char* tag) {
    const int n = (int)idx.size();
    std::vector<sgp_problem> pr(n);
    std::vector<float*> fs(n);
    std::vector<const float*> f0s(n);
    std::vector<sgp_report> reps(n);
    int seen[4] = {0, 0, 0, 0};
    std::vector<int> expect(n);
    for (int t = 0; t < n; ++t) {
      Item& it = items[idx[t]];
      pr[t] = sgp_problem{it.g, it.psf, nullptr, &it.b, 1, it.n, it.n, it.n, it.n, 0, 0, 0};
      fs[t] = it.f;
      f0s[t] = it.f0;
      int s = 0;
      while (sizes[s] != it.n) ++s;
      const int b = seen[s]++;  // item index inside its size group
      const int tg = sgp::shim_target(b);
      expect[t] = tg < max_iter ? tg : max_iter;
    }
    sgp_params p;
    sgp_params_init(&p);
    p.max_iter = max_iter;
    p.stop = SGP_STOP_DISCREPANCY | SGP_STOP_CONV;
    p.tol = 1e-7;
    if (warm) p.init = SGP_INIT_WARM;
    const int rc = sgp_batch_deconv(1, pr.data(), n, fs.data(), warm ? f0s.data() : nullptr, &p, reps.data(), nullptr);
    int wrong = 0;
    for (int t = 0; t < n; ++t) wrong += reps[t].iters != expect[t];
    printf("%-18s n=%3d max_iter=%4d rc=%d wrong=%d\n", tag, n, max_iter, rc, wrong);
    if (rc < 0 || wrong) ++bad;
  };
  std::vector<std::vector<int>> groups(4);
  for (int i : order)
    for (int s = 0; s < 4; ++s)
      if (items[i].n == sizes[s]) groups[s].push_back(i);
  for (auto& g : groups) run(g, false, 1, "group, 1 iteration");
  run(order, false, 3000, "flat, all");
  run(order, true, 3000, "warm, all");
  run(order, true, 3000, "warm, all");
  for (auto& g : groups) run(g, true, 3000, "warm, group");
  run(order, false, 3000, "flat, all");
  run(order, false, 60, "flat, all, cap 60");
  for (auto& g : groups) run(g, false, 40, "flat, group, cap 40");
  std::vector<int> half(order.begin(), order.begin() + order.size() / 2);
  run(half, true, 3000, "warm, half");
  run(order, true, 3000, "warm, all");
  // one problem through the stepping loop: graph replays (sgp_deconv), and
  // eager launches into the static workspace (sgp_deconv_noalloc); the
  // stand-in stops it at shim_target(0) iterations
  for (int max_iter : {1, 2, 50}) {
    Item& it = items[0];
    sgp_params p;
    sgp_params_init(&p);
    p.max_iter = max_iter;
    sgp_report r1, r2;
    const int rc1 = sgp_deconv(it.g, it.psf, nullptr, it.b, it.n, it.n, &p, it.f, &r1, nullptr);
    const int rc2 = sgp_deconv_noalloc(it.g, it.psf, nullptr, it.b, it.n, it.n, &p, it.f, &r2, nullptr);
    const int want = sgp::shim_target(0) < max_iter ? sgp::shim_target(0) : max_iter;
    printf("single max_iter=%2d rc=%d/%d iters=%d/%d want %d\n", max_iter, rc1, rc2, r1.iters, r2.iters, want);
    if (rc1 < 0 || rc2 < 0 || r1.iters != want || r2.iters != want) ++bad;
  }
  sgp_release_cache();
  for (auto& it : items) { free(it.g); free(it.psf); free(it.f); free(it.f0); }
  printf(bad ? "FAILED %d\n" : "ALL OK\n", bad);
  return bad ? 1 : 0;
}
