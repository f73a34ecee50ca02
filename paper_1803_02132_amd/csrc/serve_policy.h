// Admission policy of the request loop (tsb_server_*), as a host-only function
// of what the worker knows about its workspaces. It decides, for the oldest
// request that can be considered, which workspace serves it and which idle
// workspaces are released first. Kept free of any HIP call so that the rules
// can be checked on a host without a GPU.
//
// Rules, in order:
//   1. An idle workspace of the request's geometry whose particle buffers
//      already hold the catalogue serves it as it is.
//   2. An idle workspace of the geometry whose buffers must grow serves it
//      when the growth fits the budget.
//   3. Without room for a new workspace, a request whose geometry has a busy
//      workspace waits for that one (no create/destroy churn).
//   4. Otherwise idle workspaces are released, least recently used first
//      (other geometries before the request's own), until either the idle
//      workspace of the geometry can grow (it then serves the request) or a
//      new workspace fits in a free slot.
//   5. If nothing idle is left to release, the request waits for a busy
//      workspace to finish. A request whose own new workspace exceeds the
//      whole budget is rejected.
// A request never waits while no workspace is busy: waiting only happens when
// a running request will free a slot or bytes.
#pragma once

#include <cstdint>
#include <vector>

namespace tsb {

// Bytes of the particle buffers (bucket keys, bucketed records and the
// assignment work list) sized for a catalogue of n particles: capacity n + n/8
// (at least 1024), `stride` bytes per record, 8 bytes per work item, and one
// work item per tile plus one per kPartVisits visits of at most 8 tiles per
// particle.
inline int64_t particle_capacity(int64_t n) { return n + n / 8 > 1024 ? n + n / 8 : 1024; }
inline int64_t work_capacity(int64_t ntiles, int64_t cap, int part_visits) {
  return ntiles + (8 * cap + part_visits - 1) / part_visits + 1;
}
inline int64_t particle_buffer_bytes(int stride, int64_t ntiles, int part_visits, int64_t n) {
  const int64_t cap = particle_capacity(n);
  return cap * (4 + (int64_t)stride) + 8 * work_capacity(ntiles, cap, part_visits);
}

struct EngineView {
  bool busy = false;         // a request is running on it
  bool same_key = false;     // same plan geometry as the request
  int64_t bytes = 0;         // device bytes it holds (workspace + particle buffers)
  int64_t grow = 0;          // extra bytes its buffers need for the request (0: fits as is)
  double last_used = 0.0;    // time it last finished a request
};

enum AdmitKind { kAdmitUse = 0, kAdmitCreate = 1, kAdmitWait = 2, kAdmitReject = 3 };

struct AdmitDecision {
  int kind = kAdmitWait;
  int engine = -1;             // kAdmitUse: index into the views (before any release)
  std::vector<int> release;    // indices into the views, released in this order first
};

// need_new: bytes of a new workspace of the request's geometry with buffers
// for its catalogue; budget and max_slots as given to tsb_server_create.
inline AdmitDecision decide_admission(const std::vector<EngineView>& v, int64_t need_new, int64_t budget,
                                      int max_slots) {
  AdmitDecision d;
  int64_t used = 0;
  for (const EngineView& e : v) used += e.bytes;
  for (int i = 0; i < (int)v.size(); ++i) {
    if (v[i].busy || !v[i].same_key) continue;
    if (v[i].grow == 0 || used + v[i].grow <= budget) {   // rules 1 and 2
      d.kind = kAdmitUse;
      d.engine = i;
      return d;
    }
  }
  if (need_new > budget) {   // rule 5: can never fit, even alone
    d.kind = kAdmitReject;
    return d;
  }
  bool busy_same = false;
  for (const EngineView& e : v) busy_same = busy_same || (e.busy && e.same_key);
  int n_eng = (int)v.size();
  if (busy_same && !(n_eng < max_slots && used + need_new <= budget)) return d;   // rule 3: wait
  // rule 4: release idle workspaces, LRU, other geometries first
  std::vector<bool> gone(v.size(), false);
  auto next_victim = [&]() {
    int best = -1;
    for (int pass = 0; pass < 2 && best < 0; ++pass)
      for (int i = 0; i < (int)v.size(); ++i) {
        if (gone[i] || v[i].busy) continue;
        if ((pass == 0) == (v[i].same_key)) continue;   // pass 0: other geometries only
        if (best < 0 || v[i].last_used < v[best].last_used) best = i;
      }
    return best;
  };
  for (;;) {
    bool idle_same_left = false;
    for (int i = 0; i < (int)v.size(); ++i) {
      if (gone[i] || v[i].busy || !v[i].same_key) continue;
      if (used + v[i].grow <= budget) {
        d.kind = kAdmitUse;
        d.engine = i;
        return d;
      }
      idle_same_left = true;
    }
    // a new workspace only once no idle one of the geometry is left (one that
    // cannot grow is released first rather than kept beside a new one)
    if (!idle_same_left && n_eng < max_slots && used + need_new <= budget) {
      d.kind = kAdmitCreate;
      return d;
    }
    const int victim = next_victim();
    if (victim < 0) {   // everything left is busy: wait for one to finish
      d.kind = kAdmitWait;
      d.release.clear();
      return d;
    }
    gone[victim] = true;
    used -= v[victim].bytes;
    --n_eng;
    d.release.push_back(victim);
  }
}

}  // namespace tsb
