// C ABI (include/triposh.h): plan lifetime, buffers and the measurement sequence.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <limits>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "serve_policy.h"
#include "tsb_internal.h"

namespace tsb {

namespace {
thread_local std::string g_err;
}

void set_error(const std::string& msg) { g_err = msg; }

int fail(int code, const std::string& msg) {
  set_error(msg);
  return code;
}

namespace {

// Device allocation of n bytes counted in ``bytes``; with ``dry`` only the count.
int dalloc(void** p, int64_t n, int64_t& bytes, bool dry) {
  if (n <= 0) n = 1;
  *p = nullptr;
  if (!dry) {
    hipError_t e = hipMalloc(p, (size_t)n);
    if (e != hipSuccess) {
      *p = nullptr;
      return fail(e == hipErrorOutOfMemory ? TSB_E_NOMEM : TSB_E_DEVICE,
                  std::string("hipMalloc: ") + hipGetErrorString(e));
    }
  }
  bytes += n;
  return TSB_OK;
}

template <typename T>
int upload(T** dst, const std::vector<T>& v, int64_t& bytes, bool dry) {
  const int64_t n = (int64_t)std::max<size_t>(v.size(), 1) * (int64_t)sizeof(T);
  int rc = dalloc((void**)dst, n, bytes, dry);
  if (rc || dry) return rc;
  if (!v.empty()) TSB_HIP(hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return TSB_OK;
}

// e^{-2 pi i k/n}, k < n, rounded once from extended precision
int twiddles(void** dst, int n, bool f64, int64_t& bytes, bool dry) {
  std::vector<double> d(2 * (size_t)n);
  for (int k = 0; k < n; ++k) {
    const long double a = -2.0L * 3.14159265358979323846264338327950288L * (long double)k / (long double)n;
    d[2 * k] = (double)std::cos(a);
    d[2 * k + 1] = (double)std::sin(a);
  }
  if (f64) return upload((double**)dst, d, bytes, dry);
  std::vector<float> f(d.begin(), d.end());
  return upload((float**)dst, f, bytes, dry);
}

}  // namespace

// Where a plan's per-measurement buffers come from: device allocations
// (base == nullptr; with dry only the byte count) or consecutive 256-byte
// aligned pieces of a caller-given range [base, base + cap).
struct Carver {
  char* base = nullptr;
  int64_t cap = 0, used = 0;
  bool dry = false;
  int take(void** p, int64_t n, int64_t& bytes) {
    if (!base) return dalloc(p, n, bytes, dry);
    if (n <= 0) n = 1;
    used = (used + 255) / 256 * 256;
    if (used + n > cap) {
      *p = nullptr;
      used += n;
      return TSB_E_NOMEM;   // the caller reports the size it needed
    }
    *p = base + used;
    used += n;
    bytes += n;
    return TSB_OK;
  }
};

// The buffers one measurement reads and writes (grids, pass buffers, spectra,
// fields, bucketing, split-tile sums, partial sums, results), in one fixed
// order. Constant tables and the box-mode transform of y_L^M*(x^_node) are not
// among them. P.heavy_slots must already be set when carving from a range.
int carve_workspace(Plan& P, Carver& cv, int64_t& B) {
  const int64_t c = P.precision == TSB_FP64 ? 16 : 8;   // complex element
  const int64_t N = P.N, M = P.M, PG = P.PG, PF = P.PF;
  const int64_t ng = (int64_t)P.grids.size();
  const int64_t nbc = P.copies * ng;
  const int64_t nf = (int64_t)P.nb * (int64_t)P.fkinds.size();
  int rc;
#define ALLOC(ptr, n) \
  if ((rc = cv.take((void**)&(ptr), (n), B))) return rc
  ALLOC(P.d_grid, nbc * N * N * N * c);
  const int64_t PGs = pad_line(PG), PFs = pad_line(PF);
  ALLOC(P.d_t1, nbc * N * N * PGs * c);
  ALLOC(P.d_t2, nbc * N * PG * PGs * c);
  ALLOC(P.d_t3, combine_fusable((int)N) ? 0 : nbc * PG * PG * PG * c);   // x-pass output before combine_kernel
  ALLOC(P.d_spec, ng * PG * PG * PG * c);
  ALLOC(P.d_dcube, PF * PF * PF * c);
  const int64_t nv = (int64_t)P.sn_vlm.size();   // the 3PCF shot noise's two-point spectra (zero-separation bin)
  ALLOC(P.d_u1, std::max(std::max(nf * PF * PFs * M, ng * PG * PGs * M), nv * PG * PGs * M) * c);
  ALLOC(P.d_u2, std::max(std::max(nf * PFs * M * M, ng * PGs * M * M), nv * PGs * M * M) * c);
  ALLOC(P.d_fields, ((P.fused ? 0 : nf) + ng) * M * M * M * c);
  const int64_t ntiles = (int64_t)P.NT * P.NT * P.NT;
  P.nbk = assign_bucket_keys(P);
  ALLOC(P.d_bk_count, (P.nbk + 2) * 4);   // counts, then the heavy-slot and extra-part counters
  ALLOC(P.d_bk_start, (P.nbk + 1) * 4);
  ALLOC(P.d_scan_part, ((P.nbk + kScanChunk - 1) / kScanChunk + 1) * 4);
  ALLOC(P.d_tile_hslot, ntiles * 4);
  if (!cv.base) P.heavy_slots = assign_max_heavy(P, B);
  ALLOC(P.d_heavy_tile, (int64_t)P.heavy_slots * 4);
  ALLOC(P.d_heavy, assign_heavy_bytes(P));
  ALLOC(P.d_scal, (int64_t)sizeof(DevScalars));
  ALLOC(P.d_sum_partials, std::max<int64_t>(std::max<int64_t>(ntiles, 8 * 512), 512 * (int64_t)P.chans.size()) * 8);
  ALLOC(P.d_partials, (int64_t)P.red_wg * std::max<int64_t>((int64_t)P.outs.size(), 1) * 8);
  ALLOC(P.d_B, std::max<int64_t>((int64_t)P.outs.size(), 1) * 8);
#undef ALLOC
  return TSB_OK;
}

int plan_alloc(Plan& P, bool dry) {
  const int64_t c = P.precision == TSB_FP64 ? 16 : 8;   // complex element
  const int64_t N = P.N, PG = P.PG;
  const int64_t ng = (int64_t)P.grids.size();
  int64_t& B = P.bytes;
  int rc;
  Carver cv;
  cv.dry = dry;
  if ((rc = carve_workspace(P, cv, B))) return rc;
  // split-tile slots start at zero; the conversion kernel clears each slot it reads
  if (!dry) TSB_HIP(hipMemset(P.d_heavy, 0, (size_t)assign_heavy_bytes(P)));
  if (P.box_mode && P.los_kind == TSB_LOS_LOCAL && (rc = dalloc(&P.d_yspec, ng * PG * PG * PG * c, B, dry)))
    return rc;
  if (P.estimator != TSB_BISPECTRUM &&
      (rc = dalloc(&P.d_kslot, (int64_t)P.nb * (int64_t)P.fkinds.size() * P.PF * P.PF * P.PF * c, B, dry)))
    return rc;
  (void)N;
  const bool f64 = P.precision == TSB_FP64;
  if ((rc = twiddles(&P.d_tw_n, P.N, f64, B, dry))) return rc;
  if ((rc = twiddles(&P.d_tw_m, P.M, f64, B, dry))) return rc;
  if ((rc = upload(&P.d_bin_lut, P.bin_lut, B, dry))) return rc;
  {
    std::vector<int> r2(std::max(P.nb, 1), -1);   // -1: a bin with no mode
    for (size_t n2 = 0; n2 < P.bin_lut.size(); ++n2)
      if (P.bin_lut[n2] >= 0) r2[P.bin_lut[n2]] = (int)n2;
    if ((rc = upload(&P.d_bin_r2, r2, B, dry))) return rc;
  }
  {
    // combine-step tables (eq. 39 and the interlace phase, per axis)
    std::vector<double> tab(3 * (size_t)PG);
    for (int64_t j = 0; j < PG; ++j) {
      const long double n = (long double)(j - P.RG), x = n / (long double)N;
      long double w = 1.0L;
      if (j != P.RG) {
        const long double sc = std::sin((long double)M_PI * x) / ((long double)M_PI * x);
        for (int k = 0; k < P.p; ++k) w *= sc;
      }
      tab[j] = (double)(1.0L / w);
      tab[PG + j] = (double)std::cos((long double)M_PI * x);
      tab[2 * PG + j] = (double)std::sin((long double)M_PI * x);
    }
    if ((rc = upload(&P.d_axis_tab, tab, B, dry))) return rc;
  }
  if ((rc = upload(&P.d_fkinds, P.fkinds, B, dry))) return rc;
  if ((rc = upload(&P.d_fcomp, P.fcomp, B, dry))) return rc;
  if ((rc = upload(&P.d_gcomp, P.gcomp, B, dry))) return rc;
  if ((rc = upload(&P.d_terms, P.terms, B, dry))) return rc;
  if ((rc = upload(&P.d_qgroups, P.qgroups, B, dry))) return rc;
  if ((rc = upload(&P.d_outs, P.outs, B, dry))) return rc;
  if ((rc = upload(&P.d_out_norm, P.out_norm, B, dry))) return rc;
  if ((rc = upload(&P.d_f2idx, P.f2idx, B, dry))) return rc;
  if (P.shot_noise) {
    // shot noise (Sec. 4.2, eqs. 44-46): second spectra, H spectra, the cube of
    // ones, scalars, the shell mode list, alias sums and term combos
    const int64_t g3 = ng * PG * PG * PG * c;
    if ((rc = dalloc((void**)&P.d_scal_n, (int64_t)sizeof(DevScalars), B, dry))) return rc;
    if ((rc = dalloc(&P.d_nspec, g3, B, dry))) return rc;
    if ((rc = dalloc(&P.d_hspec, g3, B, dry))) return rc;
    if ((rc = dalloc((void**)&P.d_sbar, std::max<int64_t>((int64_t)P.chans.size(), 1) * 8, B, dry))) return rc;
    if ((rc = dalloc((void**)&P.d_Braw, std::max<int64_t>((int64_t)P.outs.size(), 1) * 8, B, dry))) return rc;
    if ((rc = dalloc((void**)&P.d_ssums, std::max<int64_t>((int64_t)P.sn_combos.size() * P.nb * 2, 1) * 8, B, dry)))
      return rc;
    const int64_t pf3 = P.estimator == TSB_BISPECTRUM ? (int64_t)P.PF * P.PF * P.PF : 0;
    if (pf3 == 0) {   // (the 3PCF's term needs no unit shell fields)
    } else if (P.precision == TSB_FP64) {
      std::vector<double> ones(2 * pf3, 0.0);
      for (int64_t i = 0; i < pf3; ++i) ones[2 * i] = 1.0;
      if ((rc = upload((double**)&P.d_ucube, ones, B, dry))) return rc;
    } else {
      std::vector<float> ones(2 * pf3, 0.0f);
      for (int64_t i = 0; i < pf3; ++i) ones[2 * i] = 1.0f;
      if ((rc = upload((float**)&P.d_ucube, ones, B, dry))) return rc;
    }
    if ((rc = upload(&P.d_shell_modes, P.sn_mode_list, B, dry))) return rc;
    if ((rc = upload(&P.d_shell_start, P.sn_mode_start, B, dry))) return rc;
    if ((rc = upload(&P.d_cw2_tab, P.sn_alias, B, dry))) return rc;
    if ((rc = upload(&P.d_sn_combos, P.sn_combos, B, dry))) return rc;
    if (!P.sn_vlm.empty()) {
      const int64_t nv = (int64_t)P.sn_vlm.size();
      if ((rc = upload(&P.d_sn_combo_v, P.sn_combo_v, B, dry))) return rc;
      if ((rc = dalloc(&P.d_vspec, nv * (int64_t)P.PF * P.PF * P.PF * c, B, dry))) return rc;
      if ((rc = dalloc(&P.d_vfields, nv * (int64_t)P.M * P.M * P.M * c, B, dry))) return rc;
    }
  }
  return TSB_OK;
}

void plan_free(Plan& P) {
  for (int st = 0; st < kNumStages; ++st)
    for (int k = 0; k < 2; ++k)
      if (P.ev[st][k]) (void)hipEventDestroy(P.ev[st][k]);
  if (P.graph_exec) (void)hipGraphExecDestroy(P.graph_exec);
  if (P.cap_stream) (void)hipStreamDestroy(P.cap_stream);
  if (P.own_stream) (void)hipStreamDestroy(P.own_stream);
  if (P.h_res) (void)hipHostFree(P.h_res);
  P.graph_exec = nullptr;
  P.cap_stream = P.own_stream = nullptr;
  P.h_res = nullptr;
  void* ptrs[] = {P.d_grid, P.d_t1, P.d_t2, P.d_t3, P.d_spec, P.d_dcube, P.d_u1, P.d_u2, P.d_fields,
                  P.d_tw_n, P.d_tw_m, P.d_bin_lut, P.d_bin_r2, P.d_fkinds, P.d_fcomp, P.d_gcomp, P.d_terms,
                  P.d_qgroups, P.d_outs, P.d_out_norm, P.d_partials, P.d_B, P.d_scal, P.d_sum_partials,
                  P.d_bk_count, P.d_bk_start, P.d_scan_part, P.d_keys, P.d_rec,
                  P.d_f2idx, P.d_yspec, P.d_axis_tab, P.d_tile_hslot, P.d_heavy_tile,
                  P.d_heavy, P.d_work, P.d_hostcat, P.d_scal_n, P.d_nspec, P.d_hspec, P.d_ucube,
                  P.d_sbar, P.d_Braw, P.d_ssums, P.d_shell_modes, P.d_shell_start, P.d_cw2_tab,
                  P.d_sn_combos, P.d_kslot, P.d_sn_combo_v, P.d_vspec, P.d_vfields};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
}

namespace {

int ensure_particles(Plan& P, int64_t n) {
  if (n <= P.particle_cap && P.d_rec) return TSB_OK;   // (buffers exist even for an empty catalogue)
  if (n > 2147483647LL) return fail(TSB_E_UNSUPPORTED, "more than 2^31-1 particles");
  const int64_t per = 4 + record_stride(P);   // key, record
  for (void* p : {(void*)P.d_keys, P.d_rec, P.d_work})
    if (p) (void)hipFree(p);
  P.d_keys = nullptr;
  P.d_rec = P.d_work = nullptr;
  P.bytes -= per * P.particle_cap + 8 * P.work_cap;
  P.particle_cap = P.work_cap = 0;
  const int64_t cap = particle_capacity(n);   // the sizing the server's admission assumes
  const int64_t wcap = assign_work_cap(P, cap);
  int rc;
  if ((rc = dalloc((void**)&P.d_keys, cap * 4, P.bytes, false))) return rc;
  if ((rc = dalloc(&P.d_rec, cap * record_stride(P), P.bytes, false))) return rc;
  if ((rc = dalloc(&P.d_work, wcap * 8, P.bytes, false))) return rc;
  P.particle_cap = cap;
  P.work_cap = wcap;
  ++P.particle_gen;   // buffers moved: a captured graph is stale
  return TSB_OK;
}

// Box mode with a local LOS: transform y_L^M*(x^_node) once (same passes and
// combination as the data) so that each measurement subtracts the mean term
// in spectrum space.
int init_yspec(Plan& P) {
  if (!P.d_yspec) return TSB_OK;
  int rc;
  hipStream_t s = nullptr;
  P.yspec_ready = false;
  if ((rc = run_ynode_fill(P, s))) return rc;
  if ((rc = run_forward(P, s))) return rc;
  const int64_t c = P.precision == TSB_FP64 ? 16 : 8;
  const int64_t bytes = (int64_t)P.grids.size() * P.PG * P.PG * P.PG * c;
  TSB_HIP(hipMemcpyAsync(P.d_yspec, P.d_spec, (size_t)bytes, hipMemcpyDeviceToDevice, s));
  TSB_HIP(hipStreamSynchronize(s));
  P.yspec_ready = true;
  return TSB_OK;
}

int check_catalog(const tsb_catalog* c, const char* what) {
  if (!c) return fail(TSB_E_ARG, std::string(what) + " catalogue is NULL");
  if (c->n < 0) return fail(TSB_E_ARG, std::string(what) + " catalogue has n < 0");
  if (c->on_device != 0 && c->on_device != 1)
    return fail(TSB_E_ARG, std::string(what) + " catalogue: on_device must be 0 (host) or 1 (device)");
  if (c->n > 0 && (!c->x || !c->y || !c->z))
    return fail(TSB_E_ARG, std::string(what) + " catalogue has NULL positions");
  return TSB_OK;
}

// A device catalogue's arrays must be device memory of the plan's device (a
// host pointer read by a kernel would fault the GPU).
int check_device_arrays(const Plan& P, const tsb_catalog* c, const char* what) {
  if (c->n == 0) return TSB_OK;
  for (const float* p : {c->x, c->y, c->z, c->w, c->nbar}) {
    if (!p) continue;
    hipPointerAttribute_t at{};
    const hipError_t e = hipPointerGetAttributes(&at, p);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(TSB_E_ARG, std::string(what) + " catalogue: on_device = 1 but an array is not device memory");
    }
    if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged)
      return fail(TSB_E_ARG, std::string(what) + " catalogue: on_device = 1 but an array is not device memory");
    if (at.device != P.device)
      return fail(TSB_E_ARG, std::string(what) + " catalogue: arrays on another device than the plan's");
  }
  return TSB_OK;
}

// Host catalogues: copy the arrays into the plan's buffers on stream s and
// describe the copies as a device catalogue. Slot 0 holds the data, slot 1 the
// randoms, each [5][cap] floats (x, y, z, w, nbar).
int stage_host_catalogs(Plan& P, const tsb_catalog* in[2], tsb_catalog out[2], hipStream_t s) {
  int64_t need = 0;
  for (int k = 0; k < 2; ++k)
    if (in[k] && !in[k]->on_device) need = std::max(need, in[k]->n);
  if (need > P.hostcat_cap) {
    if (P.d_hostcat) TSB_HIP(hipFree(P.d_hostcat));
    P.bytes -= 2 * 5 * 4 * P.hostcat_cap;
    P.d_hostcat = nullptr;
    P.hostcat_cap = 0;
    const int64_t cap = need + need / 8;
    int rc = dalloc(&P.d_hostcat, 2 * 5 * 4 * cap, P.bytes, false);
    if (rc) return rc;
    P.hostcat_cap = cap;
  }
  for (int k = 0; k < 2; ++k) {
    if (!in[k]) continue;
    out[k] = *in[k];
    if (in[k]->on_device) continue;
    float* base = (float*)P.d_hostcat + (int64_t)k * 5 * P.hostcat_cap;
    const float* src[5] = {in[k]->x, in[k]->y, in[k]->z, in[k]->w, in[k]->nbar};
    const float** dst[5] = {&out[k].x, &out[k].y, &out[k].z, &out[k].w, &out[k].nbar};
    for (int a = 0; a < 5 && in[k]->n > 0; ++a) {   // (an empty catalogue is never read)
      if (!src[a]) continue;                          // w / nbar absent: stays NULL
      float* d = base + a * P.hostcat_cap;
      TSB_HIP(hipMemcpyAsync(d, src[a], (size_t)in[k]->n * 4, hipMemcpyHostToDevice, s));
      *dst[a] = d;
    }
    out[k].on_device = 1;
  }
  return TSB_OK;
}

int set_device(const Plan& P) {
  int cur = -1;
  TSB_HIP(hipGetDevice(&cur));
  if (cur != P.device) return fail(TSB_E_ARG, "the plan belongs to another device than the current one");
  return TSB_OK;
}

// Weights and bucketing of a measurement. Host catalogues are copied into the
// plan's buffers first (described in `staged`); *data_out / *rand_out (if
// given) receive the device catalogues the kernels read.
int run_front(Plan& P, const tsb_catalog* data, const tsb_catalog* rand, hipStream_t s, tsb_catalog* staged,
              const tsb_catalog** data_out, const tsb_catalog** rand_out) {
  int rc;
  if ((rc = set_device(P))) return rc;
  if ((rc = check_catalog(data, "data"))) return rc;
  if (!P.box_mode && (rc = check_catalog(rand, "randoms"))) return rc;
  if (data->on_device && (rc = check_device_arrays(P, data, "data"))) return rc;
  if (!P.box_mode && rand->on_device && (rc = check_device_arrays(P, rand, "randoms"))) return rc;
  if (!data->on_device || (!P.box_mode && !rand->on_device)) {
    const tsb_catalog* in[2] = {data, P.box_mode ? nullptr : rand};
    if ((rc = stage_host_catalogs(P, in, staged, s))) return rc;
    data = &staged[0];
    if (!P.box_mode) rand = &staged[1];
  }
  const int64_t ntot = data->n + (P.box_mode ? 0 : rand->n);
  if ((rc = ensure_particles(P, ntot))) return rc;
  if ((rc = run_prep(P, data, P.box_mode ? nullptr : rand, s))) return rc;
  if ((rc = run_assign(P, data, P.box_mode ? nullptr : rand, s))) return rc;
  if (data_out) *data_out = data;
  if (rand_out) *rand_out = rand;
  return TSB_OK;
}

int run_front(Plan& P, const tsb_catalog* data, const tsb_catalog* rand, hipStream_t s) {
  tsb_catalog staged[2];
  return run_front(P, data, rand, s, staged, nullptr, nullptr);
}

// Launches per stage in one measurement (for per-launch averages).
int64_t stage_launches(const Plan& P, int st) {
  if (st == kStReduce) return ((int64_t)P.outs.size() + 16 * kBlock - 1) / (16 * kBlock);
  return 1;
}

// After the stream has been synchronised: fold the recorded event pairs into
// the accumulators.
void collect_stage_times(Plan& P) {
  for (int st = 0; st < kNumStages; ++st) {
    if (!P.ev_pending[st]) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, P.ev[st][0], P.ev[st][1]) == hipSuccess) {
      P.stage_ms[st] += ms;
      P.stage_calls[st] += stage_launches(P, st);
    }
    P.ev_pending[st] = false;
  }
}

int check_input_flags(Plan& P, const DevScalars& h) {
  if (h.err & 1) return fail(TSB_E_INPUT, "non-finite particle position or weight");
  if (h.err & 2) return fail(TSB_E_INPUT, "survey particle outside the box");
  if (h.err & 4) return fail(TSB_E_INPUT, "particle at the observer position (LOS undefined)");
  return TSB_OK;
}

// Everything after the bucketing: the assignment's tile stages, the forward
// and inverse transforms and the reduction. Launch shapes depend only on the
// plan and its particle capacity.
int run_back(Plan& P, hipStream_t s) {
  int rc;
  if ((rc = run_assign_back(P, s))) return rc;
  if ((rc = run_forward(P, s))) return rc;
  if ((rc = run_inverse(P, s))) return rc;
  if (P.fused) {
    if (!P.outs.empty()) {
      if ((rc = run_fused(P, s))) return rc;
      if ((rc = run_reduce_final(P, s))) return rc;
    }
  } else if ((rc = run_reduce(P, s))) {
    return rc;
  }
  return TSB_OK;
}

// run_back through a graph captured once per plan, particle capacity and
// profiling state (with profiling on, the stage events are event-record nodes
// of the graph, so stage times cover the replayed launches).
int launch_back(Plan& P, hipStream_t s) {
  if (!P.use_graph || (P.prof && P.prof_graph_failed)) return run_back(P, s);
  if (!P.graph_exec || P.graph_gen != P.particle_gen || P.graph_prof != P.prof || P.graph_tune != P.tune_gen) {
    if (P.graph_exec) {
      TSB_HIP(hipGraphExecDestroy(P.graph_exec));
      P.graph_exec = nullptr;
    }
    if (!P.cap_stream) TSB_HIP(hipStreamCreateWithFlags(&P.cap_stream, hipStreamNonBlocking));
    bool pending[kNumStages];
    for (int st = 0; st < kNumStages; ++st) pending[st] = P.ev_pending[st];
    TSB_HIP(hipStreamBeginCapture(P.cap_stream, hipStreamCaptureModeThreadLocal));
    const int rc = run_back(P, P.cap_stream);
    P.graph_stages = 0;
    for (int st = 0; st < kNumStages; ++st) {
      if (P.ev_pending[st] && !pending[st]) P.graph_stages |= 1u << st;
      P.ev_pending[st] = pending[st];
    }
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(P.cap_stream, &g);
    if ((rc || e != hipSuccess || !g) && P.prof) {
      // stage events could not ride in the graph: profile with direct launches
      if (g) (void)hipGraphDestroy(g);
      (void)hipGetLastError();
      P.prof_graph_failed = true;
      for (int st = 0; st < kNumStages; ++st) P.ev_pending[st] = pending[st];
      return run_back(P, s);
    }
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess || !g) return fail(TSB_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    hipGraphExec_t ex = nullptr;
    const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return fail(TSB_E_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(ei));
    P.graph_exec = ex;
    P.graph_gen = P.particle_gen;
    P.graph_prof = P.prof;
    P.graph_tune = P.tune_gen;
  }
  TSB_HIP(hipGraphLaunch(P.graph_exec, s));
  for (int st = 0; st < kNumStages; ++st)
    if (P.graph_stages >> st & 1u) P.ev_pending[st] = true;
  return TSB_OK;
}

// Bytes per pinned result slot: the outputs and the device scalars; a
// shot-noise plan adds the raw estimator, the i = j != k term, Sbar per channel
// and the shell sums.
size_t shot_extra(const Plan& P) {
  if (!P.shot_noise) return 0;
  return (P.outs.size() * 2 + P.chans.size() + P.sn_combos.size() * P.nb * 2) * 8;
}

size_t result_stride(const Plan& P) {
  return ((P.outs.size() * 8 + sizeof(DevScalars) + shot_extra(P)) + 255) / 256 * 256;
}

// Pinned result slots; growing them waits for the plan's work to drain.
int ensure_result_slots(Plan& P, int n) {
  if (n <= P.res_slots) return TSB_OK;
  TSB_HIP(hipDeviceSynchronize());
  if (P.h_res) TSB_HIP(hipHostFree(P.h_res));
  P.h_res = nullptr;
  P.res_slots = 0;
  TSB_HIP(hipHostMalloc(&P.h_res, result_stride(P) * (size_t)n, hipHostMallocDefault));
  P.res_slots = n;
  return TSB_OK;
}

// One measurement enqueued on s; its outputs and scalars land in pinned slot
// `slot` when s reaches that point.
// The inverse transforms and the reduction of the raw estimator (eq. 41).
int run_reduction_part(Plan& P, hipStream_t s) {
  int rc;
  if ((rc = run_inverse(P, s))) return rc;
  if (P.fused) {
    if (!P.outs.empty()) {
      if ((rc = run_fused(P, s))) return rc;
      if ((rc = run_reduce_final(P, s))) return rc;
    }
  } else if ((rc = run_reduce(P, s))) {
    return rc;
  }
  return TSB_OK;
}

// A shot-noise plan's measurement, launched directly (its passes interleave
// particle-count-dependent and fixed-shape launches): the estimator's pass,
// Sbar, the w^2-weighted pass of the N fields, the k-space terms, the raw
// estimator's reduction (kept in d_Braw) and the i = j != k term's reduction.
int run_shot_measure(Plan& P, const tsb_catalog* data, const tsb_catalog* rand, hipStream_t s) {
  int rc;
  tsb_catalog staged[2];
  if ((rc = run_front(P, data, rand, s, staged, &data, &rand))) return rc;
  if ((rc = run_assign_back(P, s))) return rc;
  if ((rc = run_forward(P, s))) return rc;
  if ((rc = run_sbar(P, data, P.box_mode ? nullptr : rand, s))) return rc;
  P.wpass = 1;
  rc = run_prep(P, data, P.box_mode ? nullptr : rand, s);
  if (!rc) rc = run_assign(P, data, P.box_mode ? nullptr : rand, s);
  if (!rc) rc = run_assign_back(P, s);
  if (!rc) rc = run_forward(P, s);
  P.wpass = 0;
  if (rc) return rc;
  if ((rc = run_shot_kspace(P, s))) return rc;
  if ((rc = run_reduction_part(P, s))) return rc;
  if (!P.outs.empty())
    TSB_HIP(hipMemcpyAsync(P.d_Braw, P.d_B, P.outs.size() * 8, hipMemcpyDeviceToDevice, s));
  P.spass = 1;
  if (P.d_kslot) {   // 3PCF: the H fields, then the sum over separation vectors
    rc = run_inverse(P, s);
    if (!rc) rc = run_separation_shot(P, s);
  } else {
    rc = run_reduction_part(P, s);
  }
  P.spass = 0;
  return rc;
}

int enqueue_measure(Plan& P, const tsb_catalog* data, const tsb_catalog* rand, hipStream_t s, int slot) {
  int rc;
  if (slot < 0 || slot >= P.res_slots) return fail(TSB_E_ARG, "result slot out of range");
  if (P.shot_noise) {
    if ((rc = run_shot_measure(P, data, rand, s))) return rc;
  } else {
    if ((rc = run_front(P, data, rand, s))) return rc;
    if ((rc = launch_back(P, s))) return rc;
  }
  char* base = (char*)P.h_res + result_stride(P) * (size_t)slot;
  const size_t no = P.outs.size() * 8;
  if (!P.outs.empty()) TSB_HIP(hipMemcpyAsync(base, P.d_B, no, hipMemcpyDeviceToHost, s));
  TSB_HIP(hipMemcpyAsync(base + no, P.d_scal, sizeof(DevScalars), hipMemcpyDeviceToHost, s));
  if (P.shot_noise) {
    char* x = base + no + sizeof(DevScalars);
    if (!P.outs.empty()) TSB_HIP(hipMemcpyAsync(x, P.d_Braw, no, hipMemcpyDeviceToHost, s));
    TSB_HIP(hipMemcpyAsync(x + no, P.d_sbar, P.chans.size() * 8, hipMemcpyDeviceToHost, s));
    if (!P.sn_combos.empty())
      TSB_HIP(hipMemcpyAsync(x + no + P.chans.size() * 8, P.d_ssums, P.sn_combos.size() * P.nb * 16,
                             hipMemcpyDeviceToHost, s));
  }
  return TSB_OK;
}

// After the slot's copies completed: input checks and the scatter into the
// caller's [n_mult][nb][nb] array (NaN where no pair was computed).
int finish_measure(Plan& P, int slot, double* B_out, double* I_out, double* alpha_out) {
  const char* base = (const char*)P.h_res + result_stride(P) * (size_t)slot;
  const double* hb = (const double*)base;
  DevScalars h;
  std::memcpy(&h, base + P.outs.size() * 8, sizeof(h));
  int rc;
  if ((rc = check_input_flags(P, h))) return rc;
  if (!(h.I > 0.0) || !std::isfinite(h.I))
    return fail(TSB_E_INPUT, "the normalisation I is not positive (no weighted particles or randoms): B is undefined");
  const size_t nbb = (size_t)P.nb * P.nb;
  if (P.shot_noise) {
    // slot layout: S_ij (the last reduction), scalars, raw B, Sbar, shell sums
    const char* x = base + P.outs.size() * 8 + sizeof(DevScalars);
    const double* braw = (const double*)x;
    const double* sbar = braw + P.outs.size();
    const double* sums = sbar + P.chans.size();
    shot_finish(P, sbar, sums, braw, hb, h.I, B_out);
  } else {
    for (size_t i = 0; i < P.mult.size() * nbb; ++i) B_out[i] = std::numeric_limits<double>::quiet_NaN();
    for (size_t o = 0; o < P.outs.size(); ++o) {
      const OutEntry& e = P.outs[o];
      B_out[(size_t)e.mu * nbb + (size_t)e.b1 * P.nb + e.b2] = hb[o];
    }
  }
  if (I_out) *I_out = h.I;
  if (alpha_out) *alpha_out = h.alpha;
  return TSB_OK;
}

}  // namespace

}  // namespace tsb

using namespace tsb;

struct tsb_plan {
  Plan p;
  // the request the plan was created from (a server clones it); bins.edges
  // points into `edges`
  tsb_grid grid{};
  tsb_los los{};
  tsb_kbins bins{};
  std::vector<double> edges;
  std::vector<tsb_multipole> mult;
  tsb_options opts{};
};

// Copy a request into a plan handle (the edges array is owned by the handle).
static void keep_request(tsb_plan& h, const tsb_grid* grid, const tsb_los* los, const tsb_kbins* bins,
                         const tsb_multipole* multipoles, int32_t n_multipoles, const tsb_options* options) {
  h.grid = *grid;
  h.los = *los;
  h.bins = *bins;
  h.edges.clear();
  if (bins->edges) h.edges.assign(bins->edges, bins->edges + bins->n_bins + 1);
  h.bins.edges = h.edges.empty() ? nullptr : h.edges.data();
  h.mult.assign(multipoles, multipoles + n_multipoles);
  h.opts = *options;
}

extern "C" {

const char* tsb_last_error(void) { return g_err.c_str(); }

static int copy_request(Plan& P, const tsb_grid* grid, const tsb_los* los, const tsb_kbins* bins,
                        const tsb_multipole* multipoles, int32_t n_multipoles, const tsb_options* options) {
  if (!grid || !los || !bins || !multipoles || !options) return fail(TSB_E_ARG, "NULL argument");
  if (n_multipoles < 1 || n_multipoles > 64) return fail(TSB_E_ARG, "n_multipoles must be in 1..64");
  for (int a = 0; a < 3; ++a)
    if (!(grid->box_len[a] > 0) || !std::isfinite(grid->box_len[a])) return fail(TSB_E_ARG, "box_len must be positive");
  if (grid->box_len[1] != grid->box_len[0] || grid->box_len[2] != grid->box_len[0])
    return fail(TSB_E_UNSUPPORTED, "k-shells need one fundamental frequency: box_len must be equal on the three axes");
  if (grid->n[1] != grid->n[0] || grid->n[2] != grid->n[0])
    return fail(TSB_E_UNSUPPORTED, "grids with different sizes per axis are not built yet");
  P.N = grid->n[0];
  P.L = grid->box_len[0];
  for (int a = 0; a < 3; ++a) {
    P.origin[a] = grid->origin[a];
    P.los_dir[a] = los->dir[a];
    P.observer[a] = los->observer[a];
  }
  P.p = grid->assign_p;
  P.interlace = grid->interlace;
  P.los_kind = los->kind;
  P.vertex = los->vertex;
  P.nb = bins->n_bins;
  P.kmin = bins->k_min;
  P.dk = bins->dk;
  P.edges.clear();
  if (bins->edges) {
    if (P.nb < 1 || P.nb > kMaxBins) return fail(TSB_E_ARG, "n_bins must be in 1..64");
    P.edges.assign(bins->edges, bins->edges + P.nb + 1);
  }
  P.mult.assign(multipoles, multipoles + n_multipoles);
  P.precision = options->precision;
  P.pair_mode = options->pair_mode;
  P.box_mode = options->box_mode ? 1 : 0;
  P.P0 = options->P0;
  if (options->unfused < 0 || options->unfused > 2) return fail(TSB_E_ARG, "unfused must be 0, 1 or 2");
  P.unfused = options->unfused;
  P.estimator = options->estimator;
  P.shot_noise = options->shot_noise;
  if (options->assign_tiles < 0 || options->assign_tiles > 1) return fail(TSB_E_ARG, "assign_tiles must be 0 or 1");
  P.assign_tiles = options->assign_tiles;
  return plan_build(P);
}

static void fill_info(const Plan& P, tsb_plan_info* info) {
  info->n = P.N;
  info->m = P.M;
  info->r_f = P.RF;
  info->r_g = P.RG;
  info->n_channels = (int32_t)P.chans.size();
  info->n_fields_f = (int32_t)P.fcomp.size();
  info->n_fields_g = (int32_t)P.gcomp.size();
  info->n_outputs = (int32_t)P.outs.size();
  info->n_grids = (int32_t)P.grids.size();
  info->n_fslots = (int32_t)P.fkinds.size();
  info->fused = P.fused ? (P.fused_wide ? 2 : 1) : 0;
  info->n_terms = (int32_t)P.terms.size();
  info->workspace_bytes = P.bytes;
  const double M3 = (double)P.M * P.M * P.M;
  double fl = 0.0;
  for (const OutEntry& o : P.outs) fl += 2.0 * (o.q1 - o.q0) * M3;
  fl += 3.0 * P.nb * (double)P.terms.size() * M3;
  if (P.fused) fl += (double)P.nb * P.fkinds.size() * P.M * P.M * 5.0 * P.M * std::log2((double)P.M);
  info->reduce_flops = (int64_t)fl;
  info->assign_columns = P.zcol ? 1 : 0;
}

int tsb_request_query(const tsb_grid* grid, const tsb_los* los, const tsb_kbins* bins,
                      const tsb_multipole* multipoles, int32_t n_multipoles, const tsb_options* options,
                      tsb_plan_info* info, int64_t* nmode, double* k_eff) {
  Plan P;
  int rc = copy_request(P, grid, los, bins, multipoles, n_multipoles, options);
  if (rc) return rc;
  if ((rc = plan_alloc(P, true))) return rc;
  if (info) fill_info(P, info);
  for (int b = 0; b < P.nb; ++b) {
    if (nmode) nmode[b] = P.nmode[b];
    if (k_eff) k_eff[b] = P.keff[b];
  }
  return TSB_OK;
}

int tsb_plan_query(const tsb_plan* plan, int64_t* workspace_bytes, int64_t* n_pairs_total, int64_t* nmode) {
  if (!plan) return fail(TSB_E_ARG, "NULL argument");
  const Plan& P = plan->p;
  if (workspace_bytes) *workspace_bytes = P.bytes;
  if (n_pairs_total) *n_pairs_total = (int64_t)P.outs.size();
  if (nmode)
    for (int b = 0; b < P.nb; ++b) nmode[b] = P.nmode[b];
  return TSB_OK;
}

int tsb_plan_create(const tsb_grid* grid, const tsb_los* los, const tsb_kbins* bins,
                    const tsb_multipole* multipoles, int32_t n_multipoles, const tsb_options* options,
                    tsb_plan** out) {
  if (!out) return fail(TSB_E_ARG, "NULL argument");
  *out = nullptr;
  tsb_plan* h = new (std::nothrow) tsb_plan();
  if (!h) return fail(TSB_E_NOMEM, "host allocation failed");
  Plan& P = h->p;
  int rc = copy_request(P, grid, los, bins, multipoles, n_multipoles, options);
  if (rc) {
    delete h;
    return rc;
  }
  if (hipGetDevice(&P.device) != hipSuccess) {
    delete h;
    return fail(TSB_E_DEVICE, "no HIP device");
  }
  rc = plan_alloc(P);
  if (!rc) rc = init_yspec(P);
  if (!rc) rc = run_separation_kernels(P, nullptr);
  if (rc) {
    plan_free(P);
    delete h;
    return rc;
  }
  keep_request(*h, grid, los, bins, multipoles, n_multipoles, options);
  *out = h;
  return TSB_OK;
}

int tsb_plan_destroy(tsb_plan* plan) {
  if (!plan) return TSB_OK;
  plan_free(plan->p);
  delete plan;
  return TSB_OK;
}

int tsb_plan_get_info(const tsb_plan* plan, tsb_plan_info* info) {
  if (!plan || !info) return fail(TSB_E_ARG, "NULL argument");
  fill_info(plan->p, info);
  return TSB_OK;
}

int tsb_plan_shot_noise(const tsb_plan* plan, double* S_out, double* S_ijk_out) {
  if (!plan || !S_out) return fail(TSB_E_ARG, "NULL argument");
  const Plan& P = plan->p;
  if (!P.shot_noise) return fail(TSB_E_ARG, "the plan does not subtract the shot noise");
  const size_t n = P.mult.size() * (size_t)P.nb * P.nb;
  if (P.last_S.size() != n) return fail(TSB_E_ARG, "no measurement yet");
  std::copy(P.last_S.begin(), P.last_S.end(), S_out);
  if (S_ijk_out) std::copy(P.last_Sij.begin(), P.last_Sij.end(), S_ijk_out);
  return TSB_OK;
}

int tsb_plan_nmode(const tsb_plan* plan, int64_t* nmode, double* k_eff) {
  if (!plan || !nmode) return fail(TSB_E_ARG, "NULL argument");
  const Plan& P = plan->p;
  for (int b = 0; b < P.nb; ++b) {
    nmode[b] = P.nmode[b];
    if (k_eff) k_eff[b] = P.keff[b];
  }
  return TSB_OK;
}

int tsb_plan_channel(const tsb_plan* plan, int32_t c, int32_t* L, int32_t* M, int32_t* part) {
  if (!plan || !L || !M || !part) return fail(TSB_E_ARG, "NULL argument");
  const Plan& P = plan->p;
  if (c < 0 || c >= (int32_t)P.chans.size()) return fail(TSB_E_ARG, "channel index out of range");
  *L = P.chans[c].L;
  *M = P.chans[c].M;
  *part = P.chans[c].part;
  return TSB_OK;
}

int tsb_assign(tsb_plan* plan, const tsb_catalog* data, const tsb_catalog* randoms, void* stream,
               void* grids_out) {
  if (!plan || !grids_out) return fail(TSB_E_ARG, "NULL argument");
  Plan& P = plan->p;
  hipStream_t s = (hipStream_t)stream;
  int rc;
  P.tiles_only = 1;   // the grids themselves: the tile assignment
  rc = run_front(P, data, randoms, s);
  if (!rc) rc = run_assign_back(P, s);
  P.tiles_only = 0;
  if (rc) return rc;
  if ((rc = run_unpack_grids(P, grids_out, s))) return rc;
  DevScalars h{};
  TSB_HIP(hipMemcpyAsync(&h, P.d_scal, sizeof(h), hipMemcpyDeviceToHost, s));
  TSB_HIP(hipStreamSynchronize(s));
  return check_input_flags(P, h);
}

int tsb_measure(tsb_plan* plan, const tsb_catalog* data, const tsb_catalog* randoms, void* stream,
                double* B_out, double* I_out, double* alpha_out) {
  if (!plan || !B_out) return fail(TSB_E_ARG, "NULL argument");
  Plan& P = plan->p;
  hipStream_t s = (hipStream_t)stream;
  int rc;
  if ((rc = set_device(P))) return rc;
  if ((rc = ensure_result_slots(P, 1))) return rc;
  if ((rc = enqueue_measure(P, data, randoms, s, 0))) return rc;
  TSB_HIP(hipStreamSynchronize(s));
  collect_stage_times(P);
  return finish_measure(P, 0, B_out, I_out, alpha_out);
}

int tsb_measure_batch(tsb_plan* const* plans, const tsb_catalog* const* data, const tsb_catalog* const* randoms,
                      int32_t n, void* stream, double* const* B_out, double* I_out, double* alpha_out) {
  if (n < 0 || (n > 0 && (!plans || !data || !B_out))) return fail(TSB_E_ARG, "NULL argument");
  if (n == 0) return TSB_OK;
  hipStream_t s = (hipStream_t)stream;
  // distinct plans, the slot of every item on its plan, and each plan's stream
  std::vector<Plan*> uniq;
  std::vector<int> slot(n);
  std::vector<int> count;
  for (int i = 0; i < n; ++i) {
    if (!plans[i] || !B_out[i]) return fail(TSB_E_ARG, "NULL plan or output in the batch");
    Plan* P = &plans[i]->p;
    size_t u = 0;
    while (u < uniq.size() && uniq[u] != P) ++u;
    if (u == uniq.size()) {
      uniq.push_back(P);
      count.push_back(0);
    }
    slot[i] = count[u]++;
  }
  int rc;
  for (size_t u = 0; u < uniq.size(); ++u) {
    Plan& P = *uniq[u];
    if ((rc = set_device(P))) return rc;
    if ((rc = ensure_result_slots(P, count[u]))) return rc;
    if (!P.own_stream) TSB_HIP(hipStreamCreateWithFlags(&P.own_stream, hipStreamNonBlocking));
    // particle buffers sized for the plan's largest catalogue before anything is enqueued
    int64_t most = 0;
    for (int i = 0; i < n; ++i) {
      if (&plans[i]->p != &P) continue;
      if ((rc = check_catalog(data[i], "data"))) return rc;
      int64_t nt = data[i]->n;
      if (!P.box_mode) {
        if (!randoms || (rc = check_catalog(randoms[i], "randoms"))) return rc ? rc : fail(TSB_E_ARG, "randoms missing");
        nt += randoms[i]->n;
      }
      most = std::max(most, nt);
    }
    if ((rc = ensure_particles(P, most))) return rc;
  }
  // the batch starts after the work already on the caller's stream
  hipEvent_t start;
  TSB_HIP(hipEventCreateWithFlags(&start, hipEventDisableTiming));
  TSB_HIP(hipEventRecord(start, s));
  for (Plan* P : uniq) TSB_HIP(hipStreamWaitEvent(P->own_stream, start, 0));
  int first_err = TSB_OK;
  for (int i = 0; i < n && !first_err; ++i) {
    Plan& P = plans[i]->p;
    first_err = enqueue_measure(P, data[i], randoms ? randoms[i] : nullptr, P.own_stream, slot[i]);
  }
  // the caller's stream continues after the whole batch
  for (Plan* P : uniq) {
    hipEvent_t e;
    TSB_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    TSB_HIP(hipEventRecord(e, P->own_stream));
    TSB_HIP(hipStreamWaitEvent(s, e, 0));
    TSB_HIP(hipEventDestroy(e));
  }
  for (Plan* P : uniq) TSB_HIP(hipStreamSynchronize(P->own_stream));
  TSB_HIP(hipEventDestroy(start));
  if (first_err) return first_err;
  for (Plan* P : uniq) collect_stage_times(*P);
  for (int i = 0; i < n; ++i) {
    rc = finish_measure(plans[i]->p, slot[i], B_out[i], I_out ? I_out + i : nullptr,
                        alpha_out ? alpha_out + i : nullptr);
    if (rc && !first_err) first_err = rc;
  }
  return first_err;
}

int tsb_plan_set_schedule(tsb_plan* plan, const int32_t* choice) {
  if (!plan || !choice) return fail(TSB_E_ARG, "NULL argument");
  Plan& P = plan->p;
  for (int st = 0; st < kNumStages; ++st) {
    const int c = choice[st];
    if (c != 0 && c != 8 && c != 16 && c != 32 && c != 64)
      return fail(TSB_E_ARG, "lines per workgroup must be 0 (the LDS rule), 8, 16, 32 or 64");
  }
  if (choice[kNumStages] < 0) return fail(TSB_E_ARG, "tile-kernel workgroups must be >= 0 (0: the occupancy default)");
  const int rt = choice[kNumStages + 1];
  if (rt < -1 || rt > 2) return fail(TSB_E_ARG, "reduction split must be -1, 0, 1 or 2");
  const int rb = choice[kNumStages + 2];
  if (rb != -1 && rb != 512 && rb != 1024) return fail(TSB_E_ARG, "reduction workgroup must be -1, 512 or 1024");
  if (rb == 512 && !P.fused && P.red_mfma == 8 && !reduce_pair_fits(P))
    return fail(TSB_E_ARG, "two 512-thread reduction workgroups do not fit a CU for this plan");
  for (int st = 0; st < kNumStages; ++st) P.lpw_tune[st] = choice[st];
  P.tile_wgs = choice[kNumStages];
  if (rt >= 0) P.fused_rt = rt;
  if (rb > 0 && !P.fused && P.red_mfma == 8) P.red_block = rb;
  ++P.tune_gen;
  return TSB_OK;
}

int tsb_plan_set_graphs(tsb_plan* plan, int32_t enable) {
  if (!plan) return fail(TSB_E_ARG, "NULL argument");
  plan->p.use_graph = enable != 0;
  return TSB_OK;
}

int tsb_plan_set_profiling(tsb_plan* plan, int32_t stages) {
  if (!plan) return fail(TSB_E_ARG, "NULL argument");
  Plan& P = plan->p;
  if (stages && !P.ev[0][0]) {
    for (int st = 0; st < kNumStages; ++st)
      for (int k = 0; k < 2; ++k) TSB_HIP(hipEventCreate(&P.ev[st][k]));
  }
  P.prof = (unsigned)stages & ((1u << kNumStages) - 1u);
  return TSB_OK;
}

// A tuned setting replaces the current best only when it is at least 2% faster
// (timing noise otherwise flips choices between equivalent schedules).
static constexpr double kTuneGain = 0.98;

int tsb_plan_autotune(tsb_plan* plan, const tsb_catalog* data, const tsb_catalog* randoms, void* stream,
                      int32_t reps, int32_t* choice) {
  if (!plan || !data || reps < 1) return fail(TSB_E_ARG, "bad argument");
  Plan& P = plan->p;
  hipStream_t s = (hipStream_t)stream;
  int rc;
  if ((rc = set_device(P))) return rc;
  if ((rc = ensure_result_slots(P, 1))) return rc;
  if (!P.ev[0][0]) {
    for (int st = 0; st < kNumStages; ++st)
      for (int k = 0; k < 2; ++k) TSB_HIP(hipEventCreate(&P.ev[st][k]));
  }
  std::vector<double> B((size_t)P.mult.size() * P.nb * P.nb);
  const unsigned prof_saved = P.prof;
  auto clear_times = [&]() {
    for (int st = 0; st < kNumStages; ++st) {
      P.stage_ms[st] = 0.0;
      P.stage_calls[st] = 0;
    }
  };
  auto run = [&](unsigned mask) -> int {   // one measurement with events on the stages of mask
    P.prof = mask;
    int r = enqueue_measure(P, data, randoms, s, 0);
    if (r) return r;
    TSB_HIP(hipStreamSynchronize(s));
    collect_stage_times(P);
    return finish_measure(P, 0, B.data(), nullptr, nullptr);
  };
  auto stage_time = [&](int st, double* ms) -> int {   // mean over reps (after one untimed run)
    int r = run(1u << st);
    if (r) return r;
    clear_times();
    for (int i = 0; i < reps; ++i)
      if ((r = run(1u << st))) return r;
    *ms = P.stage_calls[st] ? P.stage_ms[st] / (double)P.stage_calls[st] : 0.0;
    return TSB_OK;
  };
  // which stages launch anything, and the tile kernel's default grid
  clear_times();
  if ((rc = run((1u << kNumStages) - 1u))) {
    P.prof = prof_saved;
    return rc;
  }
  int64_t calls[kNumStages];
  for (int st = 0; st < kNumStages; ++st) calls[st] = P.stage_calls[st];
  // FFT passes of power-of-two length: lines per workgroup
  static const int kFftStages[] = {kStFwdZ, kStFwdY, kStFwdX, kStInvFX, kStInvFY, kStInvFZ,
                                   kStInvGX, kStInvGY, kStInvGZ};
  static const int kLpw[] = {0, 8, 16, 32, 64};
  for (int st : kFftStages) {
    const int len = st <= kStFwdX ? P.N : P.M;
    if (!calls[st] || (len & (len - 1)) != 0) continue;
    double best = 0.0;
    int best_lpw = 0;
    for (int c : kLpw) {
      P.lpw_tune[st] = c;
      ++P.tune_gen;
      double ms = 0.0;
      if ((rc = stage_time(st, &ms))) break;
      if (c == 0 || ms < kTuneGain * best) {   // a candidate must beat the default clearly
        best = ms;
        best_lpw = c;
      }
    }
    P.lpw_tune[st] = best_lpw;
    ++P.tune_gen;
    if (rc) break;
  }
  // persistent grid of the assignment tile kernel, around its occupancy-sized default
  if (!rc && P.tile_wgs > 0) {
    const int base = P.tile_wgs;
    static const double kScale[] = {1.0, 0.5, 0.75, 1.5, 2.0};
    double best = 0.0;
    int best_wgs = base;
    for (double f : kScale) {
      P.tile_wgs = std::max(1, (int)(base * f));
      ++P.tune_gen;
      double ms = 0.0;
      if ((rc = stage_time(kStAssign, &ms))) break;
      if (f == 1.0 || ms < kTuneGain * best) {
        best = ms;
        best_wgs = P.tile_wgs;
      }
    }
    P.tile_wgs = best_wgs;
    ++P.tune_gen;
  }
  // second phase of the one-pass reduction: (row, shell, k2) tasks, (shell, k2)
  // tasks, or every column transformed once and then the rows
  if (!rc && P.fused && P.fused_wide) {
    double best = 0.0;
    int best_rt = 1;
    for (int c : {1, 0, 2}) {
      P.fused_rt = c;
      ++P.tune_gen;
      double ms = 0.0;
      if ((rc = stage_time(kStReduce, &ms))) break;
      if (c == 1 || ms < kTuneGain * best) {
        best = ms;
        best_rt = c;
      }
    }
    P.fused_rt = best_rt;
    ++P.tune_gen;
  }
  // workgroup size of the unfused matrix-core reduction (two 512-thread
  // workgroups per CU, or one of 1024)
  if (!rc && !P.fused && P.red_mfma == 8) {
    const int base = P.red_block;
    double best = 0.0;
    int best_b = base;
    for (int c : {base, base == 512 ? 1024 : 512}) {
      if (c == 512 && !reduce_pair_fits(P)) continue;
      P.red_block = c;
      ++P.tune_gen;
      double ms = 0.0;
      if ((rc = stage_time(kStReduce, &ms))) break;
      if (c == base || ms < kTuneGain * best) {
        best = ms;
        best_b = c;
      }
    }
    P.red_block = best_b;
    ++P.tune_gen;
  }
  P.prof = prof_saved;
  clear_times();
  if (rc) return rc;
  if (choice) {
    for (int st = 0; st < kNumStages; ++st) choice[st] = P.lpw_tune[st];
    choice[kNumStages] = P.tile_wgs;
    choice[kNumStages + 1] = P.fused && P.fused_wide ? P.fused_rt : -1;
    choice[kNumStages + 2] = !P.fused && P.red_mfma == 8 ? P.red_block : -1;
  }
  return TSB_OK;
}

int tsb_plan_stage_times(tsb_plan* plan, int32_t n, double* ms, int64_t* calls, int32_t reset) {
  if (!plan || n < 0) return fail(TSB_E_ARG, "bad argument");
  Plan& P = plan->p;
  for (int st = 0; st < n && st < kNumStages; ++st) {
    if (ms) ms[st] = P.stage_ms[st];
    if (calls) calls[st] = P.stage_calls[st];
  }
  if (reset)
    for (int st = 0; st < kNumStages; ++st) {
      P.stage_ms[st] = 0.0;
      P.stage_calls[st] = 0;
    }
  return TSB_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Serving: a worker thread admits requests into slots (each slot a plan
// workspace and a stream) by HBM footprint and runs them concurrently.

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Request identity for workspace reuse: every field of the plan request,
// written field by field (no padding bytes, edges by value).
std::string request_key(const tsb_plan& t) {
  std::string k;
  auto add = [&k](const void* p, size_t n) { k.append((const char*)p, n); };
  auto i32 = [&](int32_t v) { add(&v, sizeof(v)); };
  auto f64 = [&](double v) { add(&v, sizeof(v)); };
  for (int a = 0; a < 3; ++a) {
    i32(t.grid.n[a]);
    f64(t.grid.box_len[a]);
    f64(t.grid.origin[a]);
    f64(t.los.dir[a]);
    f64(t.los.observer[a]);
  }
  i32(t.grid.assign_p);
  i32(t.grid.interlace);
  i32(t.los.kind);
  i32(t.los.vertex);
  i32(t.bins.n_bins);
  f64(t.bins.k_min);
  f64(t.bins.dk);
  i32((int32_t)t.edges.size());
  for (double e : t.edges) f64(e);
  i32(t.opts.precision);
  i32(t.opts.pair_mode);
  i32(t.opts.box_mode);
  f64(t.opts.P0);
  i32(t.opts.unfused);
  i32(t.opts.estimator);
  i32(t.opts.shot_noise);
  i32(t.opts.assign_tiles);
  for (const tsb_multipole& m : t.mult) {
    i32(m.l1);
    i32(m.l2);
    i32(m.L);
  }
  return k;
}

// The request's bins with `edges` pointing into the request's own copy.
tsb_kbins bins_of(const tsb_plan& t) {
  tsb_kbins b = t.bins;
  b.edges = t.edges.empty() ? nullptr : t.edges.data();
  return b;
}

struct Engine {
  tsb_plan* plan = nullptr;
  std::string key;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  int64_t ticket = 0;     // running request (0: idle)
  double last_used = 0.0;
};

struct Request {
  int64_t ticket = 0;
  std::string key;
  tsb_plan tmpl;          // request copy (its Plan stays empty)
  int rec_stride = 0;     // particle record bytes of the request's plan
  int64_t ntiles = 0;     // assignment tiles of the request's plan
  tsb_catalog data{}, rand{};
  bool has_rand = false;
  double* B_out = nullptr;
  double t_submit = 0.0, latency = 0.0;
  int status = TSB_OK;
  std::string message;
  bool done = false;
};

struct Server {
  int device = 0;
  int64_t budget = 0;
  int max_slots = 1;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<int64_t> queue;
  std::unordered_map<int64_t, Request> reqs;
  std::vector<Engine> engines;   // worker thread only
  bool stop = false;
  int64_t next_ticket = 1;
  int peak_running = 0;     // most requests running at once (under mu)
  int64_t released = 0;     // workspaces released to make room (under mu)
  std::thread worker;
};

int64_t engine_bytes(const Engine& e) { return e.plan ? e.plan->p.bytes : 0; }

// Bytes a measurement of n particles adds on top of a workspace (the sizing
// of ensure_particles).
int64_t particle_bytes(const Request& r, int64_t n) {
  return particle_buffer_bytes(r.rec_stride, r.ntiles, assign_part_visits(), n);
}

void destroy_engine(Engine& e) {
  if (e.plan) (void)tsb_plan_destroy(e.plan);
  if (e.done) (void)hipEventDestroy(e.done);
  if (e.stream) (void)hipStreamDestroy(e.stream);
  e = Engine{};
}

// Worker side: finish requests whose events have fired.
bool reap(Server& S) {
  bool any = false;
  for (Engine& e : S.engines) {
    if (!e.ticket) continue;
    const hipError_t q = hipEventQuery(e.done);
    if (q == hipErrorNotReady) continue;
    int rc;
    std::string msg;
    double* B_out;
    {
      std::lock_guard<std::mutex> lk(S.mu);
      B_out = S.reqs[e.ticket].B_out;
    }
    if (q != hipSuccess) {
      rc = fail(TSB_E_DEVICE, std::string("request failed on the device: ") + hipGetErrorString(q));
    } else {
      rc = finish_measure(e.plan->p, 0, B_out, nullptr, nullptr);
    }
    if (rc) msg = g_err;
    {
      std::lock_guard<std::mutex> lk(S.mu);
      Request& r = S.reqs[e.ticket];
      r.status = rc;
      r.message = msg;
      r.latency = now_s() - r.t_submit;
      r.done = true;
    }
    e.ticket = 0;
    e.last_used = now_s();
    any = true;
  }
  if (any) S.cv_done.notify_all();
  return any;
}

void finish_with_error(Server& S, int64_t ticket, int rc) {
  std::lock_guard<std::mutex> lk(S.mu);
  Request& r = S.reqs[ticket];
  r.status = rc;
  r.message = g_err;
  r.latency = now_s() - r.t_submit;
  r.done = true;
  S.cv_done.notify_all();
}

// Worker side: pick an engine for a queued request (decide_admission), after
// releasing the idle workspaces it names. Returns the engine index, -1 to
// wait, or -2 with rc set if the request can never fit.
int place(Server& S, const Request& r, int* rc) {
  const int64_t nt = r.data.n + (r.has_rand ? r.rand.n : 0);
  std::vector<EngineView> views(S.engines.size());
  for (size_t i = 0; i < S.engines.size(); ++i) {
    const Engine& e = S.engines[i];
    EngineView& v = views[i];
    v.busy = e.ticket != 0;
    v.same_key = e.key == r.key;
    v.bytes = engine_bytes(e);
    v.last_used = e.last_used;
    const int64_t cap = e.plan->p.particle_cap;
    if (v.same_key && cap < nt)
      v.grow = particle_bytes(r, nt) - (cap > 0 ? particle_bytes(r, cap - cap / 9) : 0);
  }
  tsb_plan_info info{};
  const tsb_kbins bins = bins_of(r.tmpl);
  if (int q = tsb_request_query(&r.tmpl.grid, &r.tmpl.los, &bins, r.tmpl.mult.data(),
                                (int32_t)r.tmpl.mult.size(), &r.tmpl.opts, &info, nullptr, nullptr)) {
    *rc = q;
    return -2;
  }
  const int64_t need = info.workspace_bytes + particle_bytes(r, nt);
  const AdmitDecision d = decide_admission(views, need, S.budget, S.max_slots);
  if (d.kind == kAdmitReject) {
    *rc = fail(TSB_E_NOMEM, "request does not fit the server's HBM budget");
    return -2;
  }
  if (d.kind == kAdmitWait) return -1;
  // release in the decided order (indices refer to the views, so erase from the back)
  int use = d.engine;
  std::vector<int> rel = d.release;
  std::sort(rel.begin(), rel.end());
  for (int k = (int)rel.size() - 1; k >= 0; --k) {
    destroy_engine(S.engines[rel[k]]);
    S.engines.erase(S.engines.begin() + rel[k]);
    if (use > rel[k]) --use;
  }
  if (!rel.empty()) {
    std::lock_guard<std::mutex> lk(S.mu);
    S.released += (int64_t)rel.size();
  }
  if (d.kind == kAdmitUse) return use;
  Engine e;
  e.key = r.key;
  int q = tsb_plan_create(&r.tmpl.grid, &r.tmpl.los, &bins, r.tmpl.mult.data(),
                          (int32_t)r.tmpl.mult.size(), &r.tmpl.opts, &e.plan);
  if (!q && hipStreamCreateWithFlags(&e.stream, hipStreamNonBlocking) != hipSuccess)
    q = fail(TSB_E_DEVICE, "stream creation failed");
  if (!q && hipEventCreateWithFlags(&e.done, hipEventDisableTiming) != hipSuccess)
    q = fail(TSB_E_DEVICE, "event creation failed");
  if (q) {
    destroy_engine(e);
    *rc = q;
    return -2;
  }
  S.engines.push_back(e);
  return (int)S.engines.size() - 1;
}

// Worker side: admit queued requests in arrival order; a request that has to
// wait for memory or a slot blocks later requests that would need a new
// workspace, but not those with an idle workspace of their own geometry.
bool admit(Server& S) {
  std::vector<int64_t> order;
  {
    std::lock_guard<std::mutex> lk(S.mu);
    order.assign(S.queue.begin(), S.queue.end());
  }
  bool any = false, blocked = false;
  for (int64_t t : order) {
    Request r;
    {
      std::lock_guard<std::mutex> lk(S.mu);
      r = S.reqs[t];
    }
    bool has_idle = false;
    for (const Engine& e : S.engines) has_idle = has_idle || (!e.ticket && e.key == r.key);
    if (blocked && !has_idle) continue;
    int rc = TSB_OK;
    const int i = place(S, r, &rc);
    if (i == -1) {
      blocked = true;
      continue;
    }
    {
      std::lock_guard<std::mutex> lk(S.mu);
      S.queue.erase(std::find(S.queue.begin(), S.queue.end(), t));
    }
    any = true;
    if (i == -2) {
      finish_with_error(S, t, rc);
      continue;
    }
    Engine& e = S.engines[i];
    Plan& P = e.plan->p;
    rc = ensure_result_slots(P, 1);
    if (!rc) rc = enqueue_measure(P, &r.data, r.has_rand ? &r.rand : nullptr, e.stream, 0);
    if (!rc && hipEventRecord(e.done, e.stream) != hipSuccess) rc = fail(TSB_E_DEVICE, "event record failed");
    if (rc) {
      (void)hipStreamSynchronize(e.stream);
      finish_with_error(S, t, rc);
      continue;
    }
    e.ticket = t;
    int running = 0;
    for (const Engine& x : S.engines) running += x.ticket != 0;
    std::lock_guard<std::mutex> lk(S.mu);
    S.peak_running = std::max(S.peak_running, running);
  }
  return any;
}

void serve(Server* S) {
  (void)hipSetDevice(S->device);
  for (;;) {
    bool progress = reap(*S);
    progress = admit(*S) || progress;
    bool running = false;
    for (const Engine& e : S->engines) running = running || e.ticket != 0;
    std::unique_lock<std::mutex> lk(S->mu);
    if (S->stop) {
      // cancel what is still queued, then leave once nothing runs
      for (int64_t t : S->queue) {
        Request& r = S->reqs[t];
        r.status = TSB_E_CANCELLED;
        r.message = "cancelled: the server was destroyed";
        r.done = true;
      }
      S->queue.clear();
      S->cv_done.notify_all();
      if (!running) break;
    }
    if (!progress) {
      if (running) S->cv_work.wait_for(lk, std::chrono::microseconds(100));
      else S->cv_work.wait_for(lk, std::chrono::milliseconds(5), [S] { return S->stop || !S->queue.empty(); });
    }
  }
  for (Engine& e : S->engines) destroy_engine(e);
  S->engines.clear();
}

}  // namespace

extern "C" {

int tsb_server_create(int64_t hbm_budget_bytes, int32_t max_slots, void** server) {
  if (!server || hbm_budget_bytes <= 0 || max_slots < 1) return fail(TSB_E_ARG, "bad argument");
  *server = nullptr;
  Server* S = new (std::nothrow) Server();
  if (!S) return fail(TSB_E_NOMEM, "host allocation failed");
  if (hipGetDevice(&S->device) != hipSuccess) {
    delete S;
    return fail(TSB_E_DEVICE, "no HIP device");
  }
  S->budget = hbm_budget_bytes;
  S->max_slots = max_slots;
  S->worker = std::thread(serve, S);
  *server = S;
  return TSB_OK;
}

int tsb_server_submit(void* server, const tsb_plan* plan, const tsb_catalog* data, const tsb_catalog* randoms,
                      double* B_out, int64_t* ticket) {
  if (!server || !plan || !data || !B_out || !ticket) return fail(TSB_E_ARG, "NULL argument");
  Server* S = (Server*)server;
  int rc;
  if ((rc = check_catalog(data, "data"))) return rc;
  const bool box = plan->p.box_mode != 0;
  if (!box && (rc = check_catalog(randoms, "randoms"))) return rc;
  Request r;
  r.tmpl.grid = plan->grid;
  r.tmpl.los = plan->los;
  r.tmpl.bins = plan->bins;
  r.tmpl.edges = plan->edges;
  r.tmpl.bins.edges = nullptr;   // bins_of() points it at r.tmpl.edges when used
  r.tmpl.mult = plan->mult;
  r.tmpl.opts = plan->opts;
  r.rec_stride = record_stride(plan->p);
  r.ntiles = (int64_t)plan->p.NT * plan->p.NT * plan->p.NT;
  r.key = request_key(r.tmpl);
  r.data = *data;
  if (!box) {
    r.rand = *randoms;
    r.has_rand = true;
  }
  r.B_out = B_out;
  r.t_submit = now_s();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return fail(TSB_E_CANCELLED, "the server is shutting down");
    r.ticket = S->next_ticket++;
    *ticket = r.ticket;
    S->reqs.emplace(r.ticket, std::move(r));
    S->queue.push_back(*ticket);
  }
  S->cv_work.notify_one();
  return TSB_OK;
}

int tsb_server_poll(void* server, int64_t ticket, int32_t* done, double* latency_s) {
  if (!server || !done) return fail(TSB_E_ARG, "NULL argument");
  Server* S = (Server*)server;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return fail(TSB_E_ARG, "unknown ticket");
  *done = it->second.done ? 1 : 0;
  if (latency_s) *latency_s = it->second.latency;
  if (it->second.done && it->second.status) {
    set_error(it->second.message);
    return it->second.status;
  }
  return TSB_OK;
}

int tsb_server_wait(void* server, int64_t ticket, double* latency_s) {
  if (!server) return fail(TSB_E_ARG, "NULL argument");
  Server* S = (Server*)server;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return fail(TSB_E_ARG, "unknown ticket");
  S->cv_done.wait(lk, [&] { return it->second.done; });
  if (latency_s) *latency_s = it->second.latency;
  if (it->second.status) {
    set_error(it->second.message);
    return it->second.status;
  }
  return TSB_OK;
}

int tsb_server_stats(void* server, int32_t* peak_running, int64_t* released) {
  if (!server) return fail(TSB_E_ARG, "NULL argument");
  Server* S = (Server*)server;
  std::lock_guard<std::mutex> lk(S->mu);
  if (peak_running) *peak_running = S->peak_running;
  if (released) *released = S->released;
  return TSB_OK;
}

int tsb_server_destroy(void* server) {
  if (!server) return TSB_OK;
  Server* S = (Server*)server;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  if (S->worker.joinable()) S->worker.join();
  delete S;
  return TSB_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Measurement without device allocation (tsb_measure_noalloc): the plan's
// constant tables stay where they are; every buffer a measurement reads and
// writes, including the particle records and the result array, is laid out in
// `scratch`, a file-scope device array of kScratchBytes that each device holds
// from the library's load to the end of the process. Host code never uses the
// array's name as an address: hipGetSymbolAddress gives each device's copy
// once, with that device current, and only that pointer reaches kernels and
// copies.

namespace tsb {

namespace {

constexpr int64_t kScratchBytes = 256LL << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// This device's copy of `scratch` (looked up once per device; the device must
// be current).
int scratch_base(int dev, char** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(TSB_E_DEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(TSB_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = (char*)p;
  }
  *out = g_scratch_ptr[dev];
  return TSB_OK;
}

// The plan fields a measurement's buffers hang on; saved before they are
// pointed into the scratch and put back afterwards.
struct WorkspaceState {
  void *grid, *t1, *t2, *t3, *spec, *dcube, *u1, *u2, *fields, *heavy, *rec, *work;
  int *bk_count, *bk_start, *scan_part, *tile_hslot, *heavy_tile, *keys;
  double *partials, *B, *sum_partials;
  DevScalars* scal;
  int64_t nbk, particle_cap, work_cap;
  unsigned prof;

  explicit WorkspaceState(const Plan& P)
      : grid(P.d_grid), t1(P.d_t1), t2(P.d_t2), t3(P.d_t3), spec(P.d_spec), dcube(P.d_dcube), u1(P.d_u1),
        u2(P.d_u2), fields(P.d_fields), heavy(P.d_heavy), rec(P.d_rec), work(P.d_work), bk_count(P.d_bk_count),
        bk_start(P.d_bk_start), scan_part(P.d_scan_part), tile_hslot(P.d_tile_hslot),
        heavy_tile(P.d_heavy_tile), keys(P.d_keys), partials(P.d_partials), B(P.d_B),
        sum_partials(P.d_sum_partials), scal(P.d_scal), nbk(P.nbk), particle_cap(P.particle_cap),
        work_cap(P.work_cap), prof(P.prof) {}

  void restore(Plan& P) const {
    P.d_grid = grid; P.d_t1 = t1; P.d_t2 = t2; P.d_t3 = t3; P.d_spec = spec; P.d_dcube = dcube;
    P.d_u1 = u1; P.d_u2 = u2; P.d_fields = fields; P.d_heavy = heavy; P.d_rec = rec; P.d_work = work;
    P.d_bk_count = bk_count; P.d_bk_start = bk_start; P.d_scan_part = scan_part;
    P.d_tile_hslot = tile_hslot; P.d_heavy_tile = heavy_tile; P.d_keys = keys; P.d_partials = partials;
    P.d_B = B; P.d_sum_partials = sum_partials; P.d_scal = scal; P.nbk = nbk; P.particle_cap = particle_cap;
    P.work_cap = work_cap; P.prof = prof;
  }
};

int measure_in_scratch(Plan& P, const tsb_catalog* data, const tsb_catalog* rand, hipStream_t s, double* B_out,
                       DevScalars* h) {
  int rc;
  char* base = nullptr;
  if ((rc = scratch_base(P.device, &base))) return rc;
  const int64_t ntot = data->n + (P.box_mode ? 0 : rand->n);
  if (ntot > 2147483647LL) return fail(TSB_E_UNSUPPORTED, "more than 2^31-1 particles");
  Carver cv;
  cv.base = base;
  cv.cap = kScratchBytes;
  int64_t bytes = 0;
  rc = carve_workspace(P, cv, bytes);
  const int64_t cap = std::max<int64_t>(ntot, 1);
  const int64_t wcap = assign_work_cap(P, cap);
  double* full = nullptr;
  if (!rc) rc = cv.take((void**)&P.d_keys, cap * 4, bytes);
  if (!rc) rc = cv.take(&P.d_rec, cap * record_stride(P), bytes);
  if (!rc) rc = cv.take(&P.d_work, wcap * 8, bytes);
  if (!rc) rc = cv.take((void**)&full, (int64_t)P.mult.size() * P.nb * P.nb * 8, bytes);
  if (rc) {
    // carve once more without a cap for the figure the message reports
    Carver need;
    need.base = base;
    need.cap = INT64_MAX;
    int64_t b2 = 0;
    (void)carve_workspace(P, need, b2);
    need.used += cap * 4 + 255 + cap * record_stride(P) + 255 + wcap * 8 + 255 +
                 (int64_t)P.mult.size() * P.nb * P.nb * 8;
    return fail(TSB_E_NOMEM, "tsb_measure_noalloc: this plan and catalogue need about " +
                                 std::to_string(need.used >> 20) + " MiB of the library's static scratch, which holds " +
                                 std::to_string(kScratchBytes >> 20) + " MiB");
  }
  P.particle_cap = cap;
  P.work_cap = wcap;
  P.prof = 0;
  // the split-tile slots start at zero (the scratch keeps whatever the last call left)
  if ((rc = run_fill_zero(P.d_heavy, assign_heavy_bytes(P), s))) return rc;
  if ((rc = run_prep(P, data, P.box_mode ? nullptr : rand, s))) return rc;
  if ((rc = run_assign(P, data, P.box_mode ? nullptr : rand, s))) return rc;
  if ((rc = run_back(P, s))) return rc;
  if ((rc = run_scatter_outputs(P, full, s))) return rc;
  TSB_HIP(hipMemcpyAsync(B_out, full, P.mult.size() * P.nb * P.nb * sizeof(double), hipMemcpyDeviceToHost, s));
  TSB_HIP(hipMemcpyAsync(h, P.d_scal, sizeof(DevScalars), hipMemcpyDeviceToHost, s));
  TSB_HIP(hipStreamSynchronize(s));
  return TSB_OK;
}

}  // namespace

}  // namespace tsb

extern "C" int tsb_measure_noalloc(tsb_plan* plan, const tsb_catalog* data, const tsb_catalog* randoms, void* stream,
                                   double* B_out, double* I_out, double* alpha_out) {
  if (!plan || !B_out) return fail(TSB_E_ARG, "NULL argument");
  Plan& P = plan->p;
  hipStream_t s = (hipStream_t)stream;
  int rc;
  if ((rc = set_device(P))) return rc;
  if ((rc = check_catalog(data, "data"))) return rc;
  if (!P.box_mode && (rc = check_catalog(randoms, "randoms"))) return rc;
  if (!data->on_device || (!P.box_mode && !randoms->on_device))
    return fail(TSB_E_ARG, "tsb_measure_noalloc takes device catalogues only (on_device = 1)");
  if (P.shot_noise) return fail(TSB_E_UNSUPPORTED, "tsb_measure_noalloc does not run shot-noise plans");
  if ((rc = check_device_arrays(P, data, "data"))) return rc;
  if (!P.box_mode && (rc = check_device_arrays(P, randoms, "randoms"))) return rc;
  const WorkspaceState saved(P);
  DevScalars h{};
  rc = measure_in_scratch(P, data, randoms, s, B_out, &h);
  saved.restore(P);
  if (rc) {
    (void)hipStreamSynchronize(s);   // nothing of this call stays in flight
    return rc;
  }
  if ((rc = check_input_flags(P, h))) return rc;
  if (!(h.I > 0.0) || !std::isfinite(h.I))
    return fail(TSB_E_INPUT, "the normalisation I is not positive (no weighted particles or randoms): B is undefined");
  if (I_out) *I_out = h.I;
  if (alpha_out) *alpha_out = h.alpha;
  return TSB_OK;
}
