// Host checks of the server's admission policy (paper_1803_02132_amd/csrc/serve_policy.h):
// named scenarios, then random ones against the policy's invariants. Exit
// status 0 when every check holds; each failure prints a line.
#include <cstdio>
#include <random>
#include <vector>

#include "serve_policy.h"

using namespace tsb;

static int failures = 0;
#define CHECK(c)                                                    \
  do {                                                              \
    if (!(c)) {                                                     \
      std::printf("FAIL line %d: %s\n", __LINE__, #c);              \
      ++failures;                                                   \
    }                                                               \
  } while (0)

static EngineView eng(bool busy, bool same, int64_t bytes, int64_t grow, double t) {
  EngineView v;
  v.busy = busy;
  v.same_key = same;
  v.bytes = bytes;
  v.grow = grow;
  v.last_used = t;
  return v;
}

int main() {
  // an idle workspace of the geometry that cannot grow while another
  // geometry's idle workspace holds the memory: release the other, then grow
  {
    std::vector<EngineView> v = {eng(false, true, 6, 3, 1.0), eng(false, false, 3, 0, 2.0)};
    AdmitDecision d = decide_admission(v, 8, 10, 4);
    CHECK(d.kind == kAdmitUse && d.engine == 0);
    CHECK(d.release.size() == 1 && d.release[0] == 1);
  }
  // the geometry's idle workspace cannot grow even alone: it is released and
  // a new one is created
  {
    std::vector<EngineView> v = {eng(false, true, 6, 6, 1.0), eng(false, false, 2, 0, 0.5)};
    AdmitDecision d = decide_admission(v, 9, 10, 4);
    CHECK(d.kind == kAdmitCreate);
    CHECK(d.release.size() == 2);
  }
  // idle workspace that fits as is
  {
    std::vector<EngineView> v = {eng(false, false, 5, 0, 1.0), eng(false, true, 5, 0, 2.0)};
    AdmitDecision d = decide_admission(v, 5, 10, 2);
    CHECK(d.kind == kAdmitUse && d.engine == 1 && d.release.empty());
  }
  // busy workspace of the geometry and no room: wait for it
  {
    std::vector<EngineView> v = {eng(true, true, 6, 0, 1.0)};
    AdmitDecision d = decide_admission(v, 6, 10, 4);
    CHECK(d.kind == kAdmitWait);
  }
  // busy workspace of the geometry but room for a second one: create
  {
    std::vector<EngineView> v = {eng(true, true, 4, 0, 1.0)};
    AdmitDecision d = decide_admission(v, 4, 10, 4);
    CHECK(d.kind == kAdmitCreate && d.release.empty());
  }
  // everything busy with other geometries: wait
  {
    std::vector<EngineView> v = {eng(true, false, 5, 0, 1.0), eng(true, false, 4, 0, 1.0)};
    AdmitDecision d = decide_admission(v, 4, 10, 4);
    CHECK(d.kind == kAdmitWait && d.release.empty());
  }
  // larger than the whole budget: reject
  {
    std::vector<EngineView> v;
    AdmitDecision d = decide_admission(v, 11, 10, 4);
    CHECK(d.kind == kAdmitReject);
  }
  // slots full of idle workspaces of other geometries: release the least
  // recently used one
  {
    std::vector<EngineView> v = {eng(false, false, 1, 0, 5.0), eng(false, false, 1, 0, 2.0)};
    AdmitDecision d = decide_admission(v, 1, 100, 2);
    CHECK(d.kind == kAdmitCreate && d.release.size() == 1 && d.release[0] == 1);
  }
  // random scenarios: the invariants
  std::mt19937_64 rng(12345);
  for (int it = 0; it < 200000; ++it) {
    const int n = (int)(rng() % 6);
    const int slots = 1 + (int)(rng() % 5);
    const int64_t budget = 10 + (int64_t)(rng() % 40);
    std::vector<EngineView> v;
    int64_t used = 0;
    for (int i = 0; i < n && i < slots; ++i) {
      const bool same = rng() % 3 == 0;
      const int64_t b = 1 + (int64_t)(rng() % 12);
      if (used + b > budget) break;
      used += b;
      v.push_back(eng(rng() % 3 == 0, same, b, same ? (int64_t)(rng() % 3 ? 0 : rng() % 15) : 0,
                      (double)(rng() % 100)));
    }
    const int64_t need = 1 + (int64_t)(rng() % 50);
    AdmitDecision d = decide_admission(v, need, budget, slots);
    bool any_busy = false;
    for (auto& e : v) any_busy = any_busy || e.busy;
    int64_t after = used;
    int count = (int)v.size();
    for (int r : d.release) {
      CHECK(r >= 0 && r < (int)v.size() && !v[r].busy);
      after -= v[r].bytes;
      --count;
    }
    if (need > budget && !(d.kind == kAdmitUse)) CHECK(d.kind == kAdmitReject);
    if (d.kind == kAdmitWait) CHECK(any_busy);   // waiting only for a running request
    if (!any_busy && need <= budget) CHECK(d.kind == kAdmitUse || d.kind == kAdmitCreate);
    if (d.kind == kAdmitCreate) {
      CHECK(count < slots);
      CHECK(after + need <= budget);
      for (size_t i = 0; i < v.size(); ++i) {   // a usable idle workspace is never bypassed
        bool released = false;
        for (int r : d.release) released = released || r == (int)i;
        if (!released && v[i].same_key && !v[i].busy) CHECK(after + v[i].grow > budget);
      }
    }
    if (d.kind == kAdmitUse) {
      CHECK(d.engine >= 0 && d.engine < (int)v.size());
      CHECK(!v[d.engine].busy && v[d.engine].same_key);
      for (int r : d.release) CHECK(r != d.engine);
      CHECK(after + v[d.engine].grow <= budget);
    }
  }
  std::printf("%s (%d failures)\n", failures ? "FAILED" : "ok", failures);
  return failures ? 1 : 0;
}
