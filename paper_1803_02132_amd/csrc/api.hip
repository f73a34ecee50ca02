// C ABI (include/triposh.h): plan lifetime, buffers and the measurement sequence.
#include <cmath>
#include <cstring>
#include <limits>
#include <new>

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

int plan_alloc(Plan& P, bool dry) {
  const int64_t c = P.precision == TSB_FP64 ? 16 : 8;   // complex element
  const int64_t N = P.N, M = P.M, PG = P.PG, PF = P.PF;
  const int64_t ng = (int64_t)P.grids.size();
  const int64_t nbc = P.copies * ng;
  const int64_t nf = (int64_t)P.nb * (int64_t)P.fkinds.size();
  int64_t& B = P.bytes;
  int rc;
#define ALLOC(ptr, n) \
  if ((rc = dalloc((void**)&(ptr), (n), B, dry))) return rc
  ALLOC(P.d_grid, nbc * N * N * N * c);
  ALLOC(P.d_t1, nbc * N * N * PG * c);
  ALLOC(P.d_t2, nbc * N * PG * PG * c);
  ALLOC(P.d_t3, nbc * PG * PG * PG * c);
  ALLOC(P.d_spec, ng * PG * PG * PG * c);
  ALLOC(P.d_dcube, PF * PF * PF * c);
  ALLOC(P.d_u1, std::max(nf * PF * PF * M, ng * PG * PG * M) * c);
  ALLOC(P.d_u2, std::max(nf * PF * M * M, ng * PG * M * M) * c);
  ALLOC(P.d_fields, ((P.fused ? 0 : nf) + ng) * M * M * M * c);
  if (P.box_mode && P.los_kind == TSB_LOS_LOCAL) ALLOC(P.d_yspec, ng * PG * PG * PG * c);
  const int64_t ntiles = (int64_t)P.NT * P.NT * P.NT;
  P.nbk = ntiles * 27;
  ALLOC(P.d_bk_count, (2 * P.nbk + 1) * 4);   // counts, cursors, heavy-slot counter
  P.d_bk_cursor = dry ? nullptr : P.d_bk_count + P.nbk;
  ALLOC(P.d_bk_start, (P.nbk + 1) * 4);
  ALLOC(P.d_scan_part, ((P.nbk + kScanChunk - 1) / kScanChunk + 1) * 4);
  ALLOC(P.d_tile_parts, ntiles * 4);
  ALLOC(P.d_tile_hslot, ntiles * 4);
  ALLOC(P.d_tile_pstart, (ntiles + 1) * 4);
  ALLOC(P.d_heavy_tile, (int64_t)assign_max_heavy() * 4);
  ALLOC(P.d_heavy, assign_heavy_bytes(P));
  ALLOC(P.d_scal, (int64_t)sizeof(DevScalars));
  ALLOC(P.d_sum_partials, std::max<int64_t>(ntiles, 4 * 512) * 8);
  ALLOC(P.d_partials, (int64_t)P.red_wg * std::max<int64_t>((int64_t)P.outs.size(), 1) * 8);
  ALLOC(P.d_B, std::max<int64_t>((int64_t)P.outs.size(), 1) * 8);
#undef ALLOC
  const bool f64 = P.precision == TSB_FP64;
  if ((rc = twiddles(&P.d_tw_n, P.N, f64, B, dry))) return rc;
  if ((rc = twiddles(&P.d_tw_m, P.M, f64, B, dry))) return rc;
  if ((rc = upload(&P.d_bin_lut, P.bin_lut, B, dry))) return rc;
  if ((rc = upload(&P.d_fkinds, P.fkinds, B, dry))) return rc;
  if ((rc = upload(&P.d_fcomp, P.fcomp, B, dry))) return rc;
  if ((rc = upload(&P.d_gcomp, P.gcomp, B, dry))) return rc;
  if ((rc = upload(&P.d_terms, P.terms, B, dry))) return rc;
  if ((rc = upload(&P.d_qgroups, P.qgroups, B, dry))) return rc;
  if ((rc = upload(&P.d_outs, P.outs, B, dry))) return rc;
  if ((rc = upload(&P.d_out_norm, P.out_norm, B, dry))) return rc;
  if ((rc = upload(&P.d_f2idx, P.f2idx, B, dry))) return rc;
  return TSB_OK;
}

void plan_free(Plan& P) {
  for (int st = 0; st < kNumStages; ++st)
    for (int k = 0; k < 2; ++k)
      if (P.ev[st][k]) (void)hipEventDestroy(P.ev[st][k]);
  void* ptrs[] = {P.d_grid, P.d_t1, P.d_t2, P.d_t3, P.d_spec, P.d_dcube, P.d_u1, P.d_u2, P.d_fields,
                  P.d_tw_n, P.d_tw_m, P.d_bin_lut, P.d_fkinds, P.d_fcomp, P.d_gcomp, P.d_terms,
                  P.d_qgroups, P.d_outs, P.d_out_norm, P.d_partials, P.d_B, P.d_scal, P.d_sum_partials,
                  P.d_bk_count, P.d_bk_start, P.d_scan_part, P.d_keys, P.d_rec,
                  P.d_f2idx, P.d_yspec, P.d_tile_parts, P.d_tile_hslot, P.d_tile_pstart, P.d_heavy_tile,
                  P.d_heavy, P.d_work};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
}

namespace {

int ensure_particles(Plan& P, int64_t n) {
  if (n <= P.particle_cap) return TSB_OK;
  if (n > 2147483647LL) return fail(TSB_E_UNSUPPORTED, "more than 2^31-1 particles");
  const int64_t per = 4 + record_stride(P);   // key, record
  for (void* p : {(void*)P.d_keys, P.d_rec, P.d_work})
    if (p) (void)hipFree(p);
  P.d_keys = nullptr;
  P.d_rec = P.d_work = nullptr;
  P.bytes -= per * P.particle_cap + 8 * P.work_cap;
  P.particle_cap = P.work_cap = 0;
  const int64_t cap = std::max<int64_t>(n + n / 8, 1024);
  const int64_t wcap = assign_work_cap(P, cap);
  int rc;
  if ((rc = dalloc((void**)&P.d_keys, cap * 4, P.bytes, false))) return rc;
  if ((rc = dalloc(&P.d_rec, cap * record_stride(P), P.bytes, false))) return rc;
  if ((rc = dalloc(&P.d_work, wcap * 8, P.bytes, false))) return rc;
  P.particle_cap = cap;
  P.work_cap = wcap;
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
  if (c->n > 0 && (!c->x || !c->y || !c->z))
    return fail(TSB_E_ARG, std::string(what) + " catalogue has NULL positions");
  return TSB_OK;
}

int set_device(const Plan& P) {
  int cur = -1;
  TSB_HIP(hipGetDevice(&cur));
  if (cur != P.device) return fail(TSB_E_ARG, "the plan belongs to another device than the current one");
  return TSB_OK;
}

int run_front(Plan& P, const tsb_catalog* data, const tsb_catalog* rand, hipStream_t s) {
  int rc;
  if ((rc = set_device(P))) return rc;
  if ((rc = check_catalog(data, "data"))) return rc;
  if (!P.box_mode && (rc = check_catalog(rand, "randoms"))) return rc;
  const int64_t ntot = data->n + (P.box_mode ? 0 : rand->n);
  if ((rc = ensure_particles(P, ntot))) return rc;
  if ((rc = run_prep(P, data, P.box_mode ? nullptr : rand, s))) return rc;
  if ((rc = run_assign(P, data, P.box_mode ? nullptr : rand, s))) return rc;
  return TSB_OK;
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

}  // namespace

}  // namespace tsb

using namespace tsb;

struct tsb_plan {
  Plan p;
};

extern "C" {

const char* tsb_last_error(void) { return g_err.c_str(); }

static int copy_request(Plan& P, const tsb_grid* grid, const tsb_los* los, const tsb_kbins* bins,
                        const tsb_multipole* multipoles, int32_t n_multipoles, const tsb_options* options) {
  if (!grid || !los || !bins || !multipoles || !options) return fail(TSB_E_ARG, "NULL argument");
  if (n_multipoles < 1 || n_multipoles > 64) return fail(TSB_E_ARG, "n_multipoles must be in 1..64");
  P.N = grid->n;
  P.L = grid->box_len;
  for (int a = 0; a < 3; ++a) {
    P.origin[a] = grid->origin[a];
    P.los_dir[a] = los->dir[a];
    P.observer[a] = los->observer[a];
  }
  P.p = grid->assign_p;
  P.interlace = grid->interlace;
  P.los_kind = los->kind;
  P.nb = bins->n_bins;
  P.kmin = bins->k_min;
  P.dk = bins->dk;
  P.mult.assign(multipoles, multipoles + n_multipoles);
  P.precision = options->precision;
  P.pair_mode = options->pair_mode;
  P.box_mode = options->box_mode ? 1 : 0;
  P.P0 = options->P0;
  P.unfused = options->unfused ? 1 : 0;
  return plan_build(P);
}

int tsb_plan_query(const tsb_grid* grid, const tsb_los* los, const tsb_kbins* bins,
                   const tsb_multipole* multipoles, int32_t n_multipoles, const tsb_options* options,
                   tsb_plan_info* info, int64_t* nmode) {
  Plan P;
  int rc = copy_request(P, grid, los, bins, multipoles, n_multipoles, options);
  if (rc) return rc;
  if ((rc = plan_alloc(P, true))) return rc;
  if (info) {
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
    info->workspace_bytes = P.bytes;
  }
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
  if (rc) {
    plan_free(P);
    delete h;
    return rc;
  }
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
  const Plan& P = plan->p;
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
  info->workspace_bytes = P.bytes;
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
  if ((rc = run_front(P, data, randoms, s))) return rc;
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
  if ((rc = run_front(P, data, randoms, s))) return rc;
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
  std::vector<double> hb(P.outs.size());
  DevScalars h{};
  if (!hb.empty()) TSB_HIP(hipMemcpyAsync(hb.data(), P.d_B, hb.size() * 8, hipMemcpyDeviceToHost, s));
  TSB_HIP(hipMemcpyAsync(&h, P.d_scal, sizeof(h), hipMemcpyDeviceToHost, s));
  TSB_HIP(hipStreamSynchronize(s));
  collect_stage_times(P);
  if ((rc = check_input_flags(P, h))) return rc;
  const size_t nbb = (size_t)P.nb * P.nb;
  for (size_t i = 0; i < P.mult.size() * nbb; ++i) B_out[i] = std::numeric_limits<double>::quiet_NaN();
  for (size_t o = 0; o < P.outs.size(); ++o) {
    const OutEntry& e = P.outs[o];
    B_out[(size_t)e.mu * nbb + (size_t)e.b1 * P.nb + e.b2] = hb[o];
  }
  if (I_out) *I_out = h.I;
  if (alpha_out) *alpha_out = h.alpha;
  return TSB_OK;
}

int tsb_plan_set_profiling(tsb_plan* plan, int32_t enable) {
  if (!plan) return fail(TSB_E_ARG, "NULL argument");
  Plan& P = plan->p;
  if (enable && !P.ev[0][0]) {
    for (int st = 0; st < kNumStages; ++st)
      for (int k = 0; k < 2; ++k) TSB_HIP(hipEventCreate(&P.ev[st][k]));
  }
  P.prof = enable != 0;
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
