// Internal declarations of the gfx950 bispectrum-multipole library.
// The public contract is include/triposh.h; everything here is private.
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/triposh.h"

namespace tsb {

constexpr int kMaxEll = 8;          // largest l1, l2, L accepted
constexpr int kMaxBins = 64;
constexpr int kBlock = 256;          // threads per workgroup of every kernel
constexpr int kScanPer = 16;         // elements per thread of the bucket scan
constexpr int kScanChunk = kBlock * kScanPer;

// ---------------------------------------------------------------------------
// error reporting

void set_error(const std::string& msg);
int fail(int code, const std::string& msg);

#define TSB_HIP(call)                                                              \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess)                                                          \
      return ::tsb::fail(TSB_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------
// plan description

// One real y-weighted density channel: weight w * Re(y_L^M*) (part 0) or
// w * Im(y_L^M*) (part 1) for M >= 0 (eq. 34). Negative M follow from
// dn_L^{-M}(x) = (-1)^M conj(dn_L^M(x)).
struct RealChannel { int L, M, part; };

// Two real channels transformed together as one complex grid (re + i im).
struct ComplexGrid { int re, im; };  // indices into channels; im = -1: none

// Input of one F slot (Sec. 4.2, eq. 42): sum over parts of
//   (fr + i fi) * y_l^m*(k^) * S(k) restricted to one shell,
// S = dn_0^0 (src < 0: the prepared F cube) or, for the first-vertex LOS,
// dn_L^M from the spectrum of complex grid src: the grid itself (smode 0),
// or the Hermitian part of its real (1) or imaginary (2) channel. m < 0 is
// allowed (y_l^-m = (-1)^m conj(y_l^m)).
struct FPart { int l, m; double fr, fi; int src, smode; };
struct FKind { int nparts; FPart part[2]; };

// A real field used by the reduction: part (0 re, 1 im) of F slot kind
// ``slot`` (F component) or of G grid ``slot`` (G component).
struct Component { int slot, part; };

// One real triple product of the expanded m-sum of eq. 41:
// coef * f1(x; b1) * f2(x; b2) * g(x).
struct Term { int mu, f1, f2, g; double coef; };

// Device-side constants of the reduction.
struct QGroup { int mu, f2, t0, t1; };        // Q_q(x;b1) = sum_{t0<=t<t1} coef f1 g
struct OutEntry { int mu, b1, b2, q0, q1; };  // B(mu,b1,b2) = sum_{q0<=q<q1} sum_x Q_q(b1) f2_q(b2)

// Scalars computed on the device during a measurement.
struct DevScalars {
  double sum_w, sum_w_ran, sum_abs, sum_abs_ran;
  double alpha, scale, inv_scale, mean_cell, I;
  double cmax;    // bound on |channel weight| of any particle (FP32 per-tile fixed point)
  int err;        // bit 0: non-finite input, bit 1: outside the box (survey),
                  // bit 2: particle on the observer
  int pad;
};

enum Stage {
  kStWeights = 0, kStBucket, kStAssign, kStFwdZ, kStFwdY, kStFwdX, kStCombine,
  kStInvFX, kStInvFY, kStInvFZ, kStInvGX, kStInvGY, kStInvGZ, kStReduce, kStReduceFinal, kNumStages
};

struct Plan {
  // request
  int N = 0;
  double L = 0, origin[3] = {0, 0, 0};
  int p = 3, interlace = 0;
  int los_kind = TSB_LOS_LOCAL;
  double los_dir[3] = {0, 0, 1}, observer[3] = {0, 0, 0};
  int nb = 0;
  double kmin = 0, dk = 0;
  std::vector<double> edges;      // explicit bin edges (n_bins + 1), empty: k_min + b dk
  std::vector<tsb_multipole> mult;
  int precision = TSB_FP32, pair_mode = TSB_PAIRS_PAPER, box_mode = 1, unfused = 0;
  int vertex = TSB_VERTEX_X3, estimator = TSB_BISPECTRUM, shot_noise = 0;
  bool g00_only = false;        // local LOS at the first or second vertex (App. B): G_0^0 is the one G field
  bool fsources = false;        // some F slot part filters a channel other than dn_0^0
  double P0 = 0;
  int device = 0;

  // derived geometry
  int M = 0;            // reduction grid
  int RF = 0, RG = 0;   // cube half-widths of F inputs and of spectra / G inputs
  int PF = 0, PG = 0;   // 2R+1
  int64_t n2maxF = 0;   // largest |n|^2 in any shell
  int64_t n2maxG = -1;  // G band limit on |n|^2 (-1: whole cube)
  int T = 8, NT = 0;    // assignment tile side and tiles per axis
  int copies = 1;       // 1 + interlace
  std::vector<int> bin_lut;       // bin of n^2 for n^2 in [0, 3 RF^2]; -1 none
  std::vector<int64_t> nmode;
  std::vector<double> keff;

  // channels, slots, terms
  std::vector<RealChannel> chans;
  std::vector<ComplexGrid> grids;
  std::vector<FKind> fkinds;
  std::vector<Component> fcomp, gcomp;
  std::vector<Term> terms;
  std::vector<QGroup> qgroups;
  std::vector<OutEntry> outs;
  std::vector<double> out_norm;   // per output: N H / (Nm1 Nm2 M^3) (divided by I on device)
  std::vector<double> mu_pref;

  // device buffers (owned)
  void* d_grid = nullptr;     // [copies][ngrid][N^3] complex
  void* d_t1 = nullptr;       // forward z-pass   [copies*ngrid][N][N][PG]
  void* d_t2 = nullptr;       // forward y-pass   [copies*ngrid][N][PG][PG]
  void* d_t3 = nullptr;       // forward x-pass   [copies*ngrid][PG][PG][PG]
  void* d_spec = nullptr;     // combined spectra [ngrid][PG^3]
  void* d_dcube = nullptr;    // dn_0^0 on the F cube [PF^3]
  void* d_u1 = nullptr;       // inverse z-pass (F then G)
  void* d_u2 = nullptr;       // inverse y-pass
  void* d_fields = nullptr;   // F slots then G slots, [nslots][M^3] complex
  void* d_tw_n = nullptr;     // twiddles e^{-2 pi i k/N}
  void* d_tw_m = nullptr;     // twiddles e^{-2 pi i k/M}
  int* d_bin_lut = nullptr;
  int* d_bin_r2 = nullptr;    // per bin: the largest |n|^2 of its modes (sparsity of the F chain)
  FKind* d_fkinds = nullptr;
  Component* d_fcomp = nullptr;
  Component* d_gcomp = nullptr;
  Term* d_terms = nullptr;
  QGroup* d_qgroups = nullptr;
  OutEntry* d_outs = nullptr;
  double* d_out_norm = nullptr;
  double* d_partials = nullptr;
  double* d_B = nullptr;
  DevScalars* d_scal = nullptr;
  // shot noise (Sec. 4.2, eqs. 44-46)
  int wpass = 0;                // 1 while the w^2-weighted fields N are assigned and transformed
  int assign_tiles = 0;         // request: 1 keeps the tile assignment (no column assignment)
  int zcol = 0;                 // measurements assign by columns, with the z transform
  int tiles_only = 0;           // 1 while the assignment grids themselves are wanted
  int zcol_pass = 0;            // set by the column assignment: the next forward transform skips its z pass
  int spass = 0;                // 1 while the i = j != k term runs the inverse transforms and reduction
  DevScalars* d_scal_n = nullptr;   // scalars of the w^2 pass
  void* d_nspec = nullptr;      // combined spectra of the N channels [ngrid][PG^3]
  void* d_hspec = nullptr;      // H spectra: dn_L^M N_0^0* - Sbar C/W^2 [ngrid][PG^3]
  void* d_ucube = nullptr;      // 1 on the F cube (the unit shell fields f_l^m) [PF^3]
  double* d_sbar = nullptr;     // Sbar per real channel [nch]
  double* d_Braw = nullptr;     // the raw estimator while the shot-noise term runs [outputs]
  double* d_ssums = nullptr;    // shell sums of y_l^m* (dn N_L^M* - Sbar C/W^2): [combo][bin] complex
  double* d_ssum_part = nullptr;   // their per-block partials
  int* d_shell_modes = nullptr;     // F-cube indices of the shell modes, bin by bin
  int* d_shell_start = nullptr;     // [n_bins + 1] offsets into d_shell_modes
  double* d_cw2_tab = nullptr;      // per stored axis mode: A_p, B_p (alias sums, eq. 45 reading)
  struct SnCombo { int l, m, L, M; };   // sum_{k in b} y_l^m*(k^) P_L^M(k)
  std::vector<SnCombo> sn_combos;
  SnCombo* d_sn_combos = nullptr;
  std::vector<double> sn_ybar;          // ybar_l^m*(b): [(l, m) index][bin] complex (re, im)
  std::vector<int> sn_ybar_index;       // (l, m) -> index into sn_ybar, l(l+1) + m
  struct SnTerm { int mu, m1, m2, M; double w3j; int cjk, cik; };   // complex terms of eq. 45 and their combos
  std::vector<SnTerm> sn_terms;
  std::vector<double> h_sn;             // host copies after a measurement: Sbar, sums, raw B, S_ij
  std::vector<double> last_S, last_Sij; // the last measurement's S and S_ij ([n_mult][nb][nb])
  std::vector<int> sn_mode_list, sn_mode_start;   // host copies of the shell mode list
  // 3PCF with an r-bin holding the zero separation: that bin, the (L, M) of
  // the two-point spectra dn N_L^M* - Sbar C/W^2 the other terms need, and
  // each combo's index among them
  int sn_zero_bin = -1;
  std::vector<SnCombo> sn_vlm;
  std::vector<int> sn_combo_v;
  void* d_vspec = nullptr;      // those two-point spectra on the F cube [nv][PF^3]
  void* d_vfields = nullptr;    // their inverse transforms [nv][M^3]
  int* d_sn_combo_v = nullptr;
  std::vector<double> sn_alias;                   // host copy of the alias-sum table
  double* d_sum_partials = nullptr;   // per-block partial sums (prep and I)
  double* d_axis_tab = nullptr;   // per stored axis mode: 1/W_axis, cos and sin of pi n/N
  void* d_kslot = nullptr;      // 3PCF: separation kernel of every F slot [nb * nkinds][PF^3]
  void* d_yspec = nullptr;      // box mode, local LOS: combined spectra of y_L^M*(x^_node) [ngrid][PG^3]
  bool yspec_ready = false;     // subtract mean * d_yspec in the combine step
  int* d_bk_count = nullptr;    // particles per (tile, reach class) bucket [nbk]
  int* d_bk_start = nullptr;    // bucket starts [nbk + 1]
  int* d_scan_part = nullptr;   // per-workgroup sums of the bucket scan
  int64_t nbk = 0;              // tiles * 27
  int* d_keys = nullptr;        // bucket key per particle
  int* d_tile_hslot = nullptr;  // heavy slot per tile or -1 [ntiles]
  int* d_heavy_tile = nullptr;  // tile of each heavy slot
  int heavy_slots = 0;          // slots of split tiles (d_heavy_tile, d_heavy)
  void* d_heavy = nullptr;      // fixed-point sums of split tiles [slot][copies][words][T^3]
  void* d_work = nullptr;       // work items (tile, part) [work_cap]
  int64_t work_cap = 0;
  int tile_wgs = 0;             // resident workgroups of the tile kernel (from the occupancy query)
  int64_t particle_gen = 0;     // bumped when particle buffers are reallocated

  // launch machinery
  bool use_graph = true;        // replay the fixed-shape part of a measurement as a graph
  hipGraphExec_t graph_exec = nullptr;
  int64_t graph_gen = -1;       // particle_gen the graph was captured with
  unsigned graph_prof = 0;      // stage mask of the event records the graph holds
  int tune_gen = 0;             // bumped whenever a launch parameter changes
  int graph_tune = 0;           // the tune_gen the graph was captured with
  int lpw_tune[kNumStages] = {};   // FFT lines per workgroup per stage (0: the LDS rule)
  uint32_t graph_stages = 0;    // stages whose events the graph records
  bool prof_graph_failed = false;   // profiling falls back to direct launches
  hipStream_t cap_stream = nullptr;   // capture stream (never executes)
  hipStream_t own_stream = nullptr;   // the plan's stream for batched measurements
  void* h_res = nullptr;        // pinned result slots: [slot][outputs doubles + DevScalars]
  int res_slots = 0;
  void* d_rec = nullptr;      // particle records in bucket order (u, channel weights), [cap][stride]
  int64_t particle_cap = 0;
  void* d_hostcat = nullptr;    // device copies of host catalogues: [2][5][hostcat_cap] float
  int64_t hostcat_cap = 0;
  int red_chunk = 64, red_wg = 1024;
  int red_mfma = 0;             // unfused FP32 reduction on the matrix cores: Q-group tiles per wavefront (0: off;
                                // 8: the wide kernel)
  int red_block = 1024;         // wide kernel: threads per workgroup, 1024 or 512 (two per CU; autotuned)
  int64_t bytes = 0;

  // fused last F pass + reduction
  bool fused = false;
  bool fused_wide = false;      // one-pass FP32 kernel (all shells of a line at once)
  int fused_bpg = 1;            // shells per group inside the fused kernel
  int fused_rt = 1;             // one-pass kernel's second phase: 1 (row, shell, k2) tasks, 0 (shell, k2)
                                // tasks, 2 columns transformed once, then the rows (autotuned)
  int nf2 = 0;                  // F components used as right factors
  std::vector<int> f2idx;       // per F component: its right-factor row or -1
  int* d_f2idx = nullptr;
  int64_t g_offset = 0;         // element offset of the G grids in d_fields

  // stage timing (HIP events on the measurement stream)
  unsigned prof = 0;            // stages bracketed by timing events (bit per stage)
  hipEvent_t ev[kNumStages][2] = {};
  bool ev_pending[kNumStages] = {};
  double stage_ms[kNumStages] = {};
  int64_t stage_calls[kNumStages] = {};
};

// Bracket a stage with events when profiling is on (errors ignored: timing
// only). Inside a stream capture the record becomes an external event node of
// the graph, so that replays record the event too.
inline void prof_record(hipEvent_t e, hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  (void)hipStreamIsCapturing(s, &cs);
  if (cs == hipStreamCaptureStatusActive) (void)hipEventRecordWithFlags(e, s, hipEventRecordExternal);
  else (void)hipEventRecord(e, s);
}
inline void prof_begin(Plan& P, int st, hipStream_t s) {
  if (((P.prof >> st) & 1u) && P.ev[st][0]) prof_record(P.ev[st][0], s);
}
inline void prof_end(Plan& P, int st, hipStream_t s) {
  if (((P.prof >> st) & 1u) && P.ev[st][1]) {
    prof_record(P.ev[st][1], s);
    P.ev_pending[st] = true;
  }
}

// Stored innermost extent of the pruned pass buffers: rows padded to 16
// elements so that groups of 16 consecutive entries start on 128-byte lines.
inline int64_t pad_line(int64_t n) { return (n + 15) / 16 * 16; }

int plan_build(Plan& P);   // host planning (plan.hip)
double three_j(int j1, int j2, int j3, int m1, int m2, int m3);   // Wigner 3j (Racah), plan.hip
std::complex<double> ylm_any(int l, int m, const double* d, const double* norm);   // y_l^m(d), any m
// (-1)^m sqrt((l-m)!/(l+m)!) at index l(l+1)/2 + m, l <= kMaxEll (45 entries)
void ylm_norm_table(double* norm);
int plan_alloc(Plan& P, bool dry = false);   // device buffers (api.hip); dry: sizes only
void plan_free(Plan& P);

// ---------------------------------------------------------------------------
// launchers (each enqueues on ``s``; returns TSB_OK or an error code)

int run_prep(Plan& P, const tsb_catalog* data, const tsb_catalog* rand, hipStream_t s);
int run_assign(Plan& P, const tsb_catalog* data, const tsb_catalog* rand, hipStream_t s);
int run_forward(Plan& P, hipStream_t s);
int run_inverse(Plan& P, hipStream_t s);
int run_separation_kernels(Plan& P, hipStream_t s);   // 3PCF: fills d_kslot
int64_t reduce_lds_bytes(const Plan& P);                // staged rows of the unfused reduction, reduce.hip
bool reduce_pair_fits(const Plan& P);                   // two 512-thread workgroups of it per CU
int run_reduce(Plan& P, hipStream_t s);
int run_reduce_final(Plan& P, hipStream_t s);
void plan_fused(Plan& P);                   // fused.hip
int run_fused(Plan& P, hipStream_t s);
int run_ynode_fill(Plan& P, hipStream_t s);
int run_assign_back(Plan& P, hipStream_t s);
bool zcol_applies(const Plan& P);      // the plan can assign by columns with the z transform
int64_t zcol_lds_bytes(const Plan& P);
int64_t assign_bucket_keys(const Plan& P);
// a measurement's assignment runs by columns (not for the w^2 fields of the
// shot noise, nor when the grids themselves are returned)
inline bool zcol_active(const Plan& P) { return P.zcol && !P.wpass && !P.tiles_only; }
int64_t assign_work_cap(const Plan& P, int64_t particles);
int assign_part_visits();   // visits per assignment work item
int record_stride(const Plan& P);
int assign_words(const Plan& P);
int64_t assign_heavy_bytes(const Plan& P);
int assign_max_heavy(const Plan& P, int64_t other_bytes);
int run_unpack_grids(Plan& P, void* out, hipStream_t s);
int run_fill_zero(void* p, int64_t bytes, hipStream_t s);        // kernel fill, bytes % 8 == 0
int run_sbar(Plan& P, const tsb_catalog* data, const tsb_catalog* rand, hipStream_t s);   // Sbar per channel
int run_shot_kspace(Plan& P, hipStream_t s);
int run_separation_shot(Plan& P, hipStream_t s);   // the 3PCF's i = j != k term (shot.hip)
// Whether the forward x pass of an N grid runs fused with the combination of
// the interlaced copies (register-FFT lengths; else a pass buffer and combine_kernel).
bool combine_fusable(int N);
bool unfused_mfma_applies(const Plan& P);   // plan.hip
// The inverse chain of nbatch complex cubes of half-width RG (G-cube layout)
// into full fields [nbatch][M^3] (fft.hip).
int run_inverse_cube(Plan& P, const void* cube, int nbatch, void* out, hipStream_t s);   // H spectra and the shell sums (shot.hip)
int shot_plan(Plan& P);                        // host tables of the shot noise (shot.hip)
void shot_finish(Plan& P, const double* sbar, const double* sums, const double* Braw, const double* Sij,
                 double I, double* B_out);      // host: S and B - S (shot.hip)
int run_scatter_outputs(Plan& P, double* full, hipStream_t s);   // [n_mult][nb][nb], NaN where not computed

// ---------------------------------------------------------------------------
// device helpers

template <typename T> struct cplx;
template <> struct cplx<float> { typedef float2 type; };
template <> struct cplx<double> { typedef double2 type; };

// Normalised harmonic y_l^m(u) for m >= 0 at a unit vector u (App. A, eq. A3),
// written without dividing by sin(theta):
//   y_l^m = (-1)^m sqrt((l-m)!/(l+m)!) Q_l^m(z) (x + i y)^m,
// with Q_l^m = d^m P_l / dz^m from the recurrence
//   Q_m^m = (2m-1)!!,  Q_{m+1}^m = (2m+1) z Q_m^m,
//   (l-m) Q_l^m = (2l-1) z Q_{l-1}^m - (l+m-1) Q_{l-2}^m.
// ``norm`` holds (-1)^m sqrt((l-m)!/(l+m)!) for (l, m) at index l*(l+1)/2 + m.
__host__ __device__ inline void ylm_pos_m(int l, int m, double x, double y, double z,
                                          const double* norm, double* re, double* im) {
  double q_mm = 1.0;
  for (int i = 1; i <= m; ++i) q_mm *= (2.0 * i - 1.0);
  double q;
  if (l == m) {
    q = q_mm;
  } else {
    double qa = q_mm, qb = (2.0 * m + 1.0) * z * q_mm;
    for (int ll = m + 2; ll <= l; ++ll) {
      double qc = ((2.0 * ll - 1.0) * z * qb - (ll + m - 1.0) * qa) / (double)(ll - m);
      qa = qb;
      qb = qc;
    }
    q = qb;
  }
  // (x + i y)^m
  double pr = 1.0, pi = 0.0;
  for (int i = 0; i < m; ++i) {
    double t = pr * x - pi * y;
    pi = pr * y + pi * x;
    pr = t;
  }
  double c = norm[l * (l + 1) / 2 + m] * q;
  *re = c * pr;
  *im = c * pi;
}

}  // namespace tsb
