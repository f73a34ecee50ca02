/*
 * triposh.h -- C ABI of the MI355X (gfx950) bispectrum-multipole library.
 *
 * Computes the decomposed bispectrum multipoles B_{l1 l2 L}(k1, k2) of a
 * weighted particle catalogue with the FFT-based estimator of Sugiyama, Saito,
 * Beutler & Seo, arXiv:1803.02132:
 *   - y-weighted density fields dn_L^M(x) = y_L^M*(x^) dn(x)       (Sec. 4.1, eq. 34)
 *   - mass assignment and W_mass deconvolution                      (Sec. 4.2, eq. 39)
 *   - F_l^m(x;k) and G_L^M(x) by inverse FFTs                       (Sec. 4.2, eq. 42)
 *   - B = H sum_{m1 m2 M} 3j (N/I) int d3x F F G                    (Sec. 4.2, eq. 41;
 *                                                                     Sec. 4.4, eq. 52)
 *   - normalisation I                                               (Sec. 4.2, eq. 37; Sec. 4.4)
 *
 * Conventions fixed by the library where the paper is silent:
 *   - grid nodes sit at origin + j * L/N (j = 0..N-1 per axis), periodic;
 *     grid coordinate u = (x - origin) * (N / L) evaluated in FP64;
 *   - assignment kernels NGP/CIC/TSC of Hockney & Eastwood (App. C);
 *   - interlacing: second grid from particles shifted by +L/(2N) per axis,
 *     combined as (D1 + e^{i pi (nx+ny+nz)/N} D2)/2 before dividing by W_mass;
 *   - k-shells [k_min + b dk, k_min + (b+1) dk) in |k| (eq. 38), membership
 *     floor((k_f sqrt(n^2) - k_min)/dk) per integer n^2 in FP64, DC excluded;
 *   - modes with an index component equal to N/2 are zero in every field;
 *   - periodic box (box_mode = 1): dn = n - nbar with nbar = sum w / V, i.e.
 *     (sum w / N^3) y_L^M*(x^_node) is subtracted at every node, the DC mode
 *     of dn_0^0 is zero, and I = (sum w)^3 / V^2;
 *   - survey (box_mode = 0): dn = data - alpha randoms with
 *     alpha = sum_data w / sum_rand w (Sec. 4.1), I = v_c sum_j (alpha R_j/v_c)^3
 *     with R the randoms assigned on the first grid;
 *   - FKP weight (Sec. 5.2, eq. 54): w = w_c / (1 + nbar P0) when P0 > 0 and
 *     the catalogue carries nbar; otherwise w = w_c.
 *
 * Every call returns 0 (TSB_OK) or a negative tsb_status; nothing throws across
 * the ABI. tsb_last_error() returns a thread-local message for the last failure.
 * All device work is enqueued on the caller's HIP stream; calls that return
 * results to host memory synchronise that stream before returning.
 * Calls on one plan must not overlap (a plan owns one workspace).
 */
#ifndef TRIPOSH_H
#define TRIPOSH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TSB_OK = 0,
  TSB_E_ARG = -1,          /* NULL pointer, size or value out of range */
  TSB_E_UNSUPPORTED = -2,  /* valid request the library does not implement */
  TSB_E_NOMEM = -3,        /* device allocation failed */
  TSB_E_INPUT = -4,        /* bad particle data: NaN/Inf position or weight,
                              survey particle outside the box, particle on the observer */
  TSB_E_DEVICE = -5,       /* a HIP call failed */
  TSB_E_BUSY = -6,         /* server: request not finished yet */
  TSB_E_CANCELLED = -7     /* server: request dropped when the server was destroyed */
} tsb_status;

enum { TSB_LOS_GLOBAL = 0, TSB_LOS_LOCAL = 1 };
enum { TSB_VERTEX_X3 = 0,        /* LOS at the vertex of the third field (Sec. 4.1, the main text) */
       TSB_VERTEX_X1 = 1,        /* LOS at the vertex of the first field (App. B) */
       TSB_VERTEX_X2 = 2 };      /* LOS at the vertex of the second field (App. B) */
enum { TSB_NGP = 1, TSB_CIC = 2, TSB_TSC = 3 };
enum { TSB_FP32 = 0, TSB_FP64 = 1 };
enum { TSB_PAIRS_PAPER = 0,      /* b1 <= b2 when l1 == l2, else every (b1, b2) (Sec. 5.2) */
       TSB_PAIRS_UPPER = 1,      /* b1 <= b2 */
       TSB_PAIRS_DIAGONAL = 2,   /* b1 == b2 (Sec. 4.4, "diagonal" measurement) */
       TSB_PAIRS_ALL = 3 };
/* Estimators. The 3PCF and the window multipoles average over the grid
 * separation vectors r = H n (H = box_len / n) whose length falls in each
 * r-bin (the configuration-space counterpart of the k-shells; the zero
 * separation, if a bin holds r = 0, enters with y_l^m = delta_l0), so that
 * zeta(b1, b2) is eq. 47 with those averages, computed in the FFT form of
 * eq. 48 with F_l^m(x; b) = (1/V) sum_k e^{ik.x} dn(k) K_l^m(k; b) and
 * K_l^m(k; b) = (1/N_r) sum_{n in b} y_l^m*(n^) e^{ik.Hn} (eq. 49 on the grid).
 * N_r and the mean |r| per bin are what tsb_plan_nmode reports for them. The
 * window multipoles need survey mode. The 3PCF shot noise is eq. 51 on the
 * grid: for r-bins without the zero separation only its i = j != k term is
 * left, on r1 = r2 bins, (N H / I)(N^3/V) sum_m 3j (-1)^{l1+l2} N_r^-2
 * sum_{n in b} y_l1^m1*(n^) y_l2^m2*(n^) H_L^M(H n) with the H field of
 * eq. 45. A bin holding r = 0 adds, on its row and column, the terms with
 * the kernel average Kbar_0^0 = N^3/(V N_r): Kbar Kbar Sbar and the two-point
 * sums (1/(V N_r)) sum_{n in b} y_l^m*(n^) v(H n), v the inverse transform of
 * dn N_L^M* - Sbar C/W^2. */
enum { TSB_BISPECTRUM = 0,       /* B_{l1 l2 L}(k1, k2) (Sec. 4.2, eq. 41) */
       TSB_3PCF = 1,             /* zeta_{l1 l2 L}(r1, r2) (Sec. 4.3, eqs. 47-48) */
       TSB_WINDOW = 2 };         /* Q_{l1 l2 L}(r1, r2) from the randoms alone (Sec. 6.1, eq. 58):
                                    randoms weighted +alpha w, galaxies only fix alpha */

/* Measurement grid (Sec. 4.2; Sec. 5.2 "Prescription"). Per-axis sizes: the
 * Nyquist frequency of axis a is pi n[a] / box_len[a] (W_mass, eq. 39). The
 * k-shells are spheres in |k|, so the library needs the same fundamental
 * frequency 2 pi / box_len[a] on every axis (equal box_len) and, when the n[a]
 * differ, every shell and the band of G below each axis' half Nyquist
 * frequency (then the reduction grid is cubic); other shapes are reported as
 * TSB_E_UNSUPPORTED. */
typedef struct {
  int32_t n[3];       /* grid points per axis: 2^a 3^b, 16 <= n <= 1024, n % 4 == 0 */
  double box_len[3];  /* side of the box per axis, > 0 */
  double origin[3];   /* position of node (0,0,0) */
  int32_t assign_p;   /* TSB_NGP, TSB_CIC or TSB_TSC: W_mass exponent p (eq. 39) */
  int32_t interlace;  /* 0 or 1 */
} tsb_grid;

/* Line of sight (Sec. 2; Sec. 4.2 local vertex x^3; Sec. 4.4 global; App. B). */
typedef struct {
  int32_t kind;        /* TSB_LOS_GLOBAL or TSB_LOS_LOCAL */
  double dir[3];       /* global: LOS direction (normalised by the library) */
  double observer[3];  /* local: observer position; the LOS of a particle is
                          the unit vector from the observer to it */
  int32_t vertex;      /* local: TSB_VERTEX_X3 (0, the paper's choice),
                          TSB_VERTEX_X1 or TSB_VERTEX_X2 (the y_L^M* weight
                          rides on the first or second field of the triangle,
                          App. B; bispectrum plans without shot noise) */
} tsb_los;

/* Bins (eq. 38). Bispectrum: k-shells [k_min + b dk, k_min + (b+1) dk) in |k|,
 * b = 0..n_bins-1, every shell below the Nyquist frequency. 3PCF and window:
 * the same rule on the separation |r| of two grid nodes (length units), every
 * bin inside half the box. With `edges` (n_bins + 1 ascending values, host
 * memory, copied at plan creation) bin b is [edges[b], edges[b+1]) and
 * k_min / dk are ignored. */
typedef struct {
  int32_t n_bins;        /* 1..64 */
  double k_min;          /* >= 0 */
  double dk;             /* > 0 */
  const double* edges;   /* NULL, or n_bins + 1 strictly increasing values >= 0 */
} tsb_kbins;

/* One multipole (l1, l2, L) (Sec. 2, eq. 11). Accepted when L is even,
 * |l1-l2| <= L <= l1+l2, l1+l2+L is even (Table 1) and l1, l2, L <= 8;
 * l1 < l2 is accepted (the transpose of (l2, l1, L)). */
typedef struct {
  int32_t l1, l2, L;
} tsb_multipole;

typedef struct {
  int32_t precision;  /* TSB_FP32: channel weights, fields, transforms and the
                         per-line products of the reduction in FP32 (see the
                         note below); TSB_FP64: FP64 throughout */
  int32_t pair_mode;  /* TSB_PAIRS_* */
  int32_t box_mode;   /* 1: periodic box without randoms; 0: survey with randoms */
  double P0;          /* FKP P0; <= 0 disables the FKP factor */
  int32_t unfused;    /* 0 (default): run the last F transform inside the
                         reduction when the plan fits, except FP32 plans whose
                         one-pass reduction would take its shells in groups and
                         whose F fields take at most 4 GiB, which write the F
                         fields and reduce them on the matrix cores (faster
                         there); 1: always write the F fields and reduce
                         separately; 2: the one-pass path whenever the plan
                         fits. The paths agree to rounding. */
  int32_t estimator;  /* TSB_BISPECTRUM, TSB_3PCF or TSB_WINDOW */
  int32_t shot_noise; /* 1 subtracts the shot noise S: the bispectrum's of Sec. 4.2
                         (eqs. 44-46: the four coincident-index terms), the
                         3PCF's of eq. 51 (third-vertex LOS, not window plans) */
  int32_t assign_tiles; /* 0 (default): box-mode FP32 plans on grids of 32, 64,
                         128 or 256 points with up to four complex grids per
                         copy assign by columns of 2 x 2 x N nodes and
                         transform each column's z lines before anything
                         reaches device memory (the grids are never stored);
                         1: always assign by tiles and store the grids. The
                         paths agree to rounding (the column path's
                         fixed-point step follows each column's visit count). */
} tsb_options;
/* FP32 plans, precisely: channel weights are computed in FP64 and stored in
 * FP32 (survey plans round each one up or down with probability given by its
 * distance to the two neighbouring FP32 values, so that the many particles
 * sharing an n-bar share no rounding error); assignment contributions are
 * rounded to 64-bit fixed point (exact integer sums; survey plans round the
 * per-tile packed sums the same unbiased way, deterministically; column plans
 * pack at a scale of each column's own, whose step grows with the column's
 * visit count); every grid, spectrum and field is FP32 (the interlace
 * combination and the W_mass division compute in FP64). The fused reduction
 * forms each Q row (a 3j-weighted sum of F G products, coefficients rounded to
 * FP32) and multiplies it with the right factor in FP32, summing the products
 * of one z-line of M cells in FP32 (matrix cores) before the line sums are
 * added in FP64; the unfused reduction forms Q in FP64, stores it in FP32 and
 * sums chunks of at most 64 cells in FP32 before FP64. The 3j symbols, H, N, N_mode,
 * k_eff, I, alpha and the final normalisation are FP64. */

/* Particle catalogue: structure of arrays owned by the caller and only read.
 * w and nbar may be NULL (w_c = 1; no FKP factor). n may be 0. With
 * on_device = 1 the arrays are device memory of the current device; with
 * on_device = 0 they are host memory, copied by the library into buffers of
 * the plan on the measurement stream (they must stay valid until the call
 * returns). */
typedef struct {
  const float* x;
  const float* y;
  const float* z;
  const float* w;
  const float* nbar;
  int64_t n;
  int32_t on_device;
} tsb_catalog;

/* Derived sizes of a plan. */
typedef struct {
  int32_t n;               /* measurement grid points along x (n[0]) */
  int32_t m;               /* reduction grid M (<= n): the estimator's sum over
                              cells is evaluated exactly on an M^3 grid when the
                              shells and G are band-limited */
  int32_t r_f;             /* largest |n_i| of any mode in any shell */
  int32_t r_g;             /* largest |n_i| of the modes G needs */
  int32_t n_channels;      /* real y-weighted density channels per grid */
  int32_t n_fields_f;      /* real F fields per shell */
  int32_t n_fields_g;      /* real G fields */
  int32_t n_outputs;       /* (multipole, b1, b2) entries computed */
  int32_t n_grids;         /* complex grids per assignment copy (two real channels each) */
  int32_t n_fslots;        /* complex F transforms per shell */
  int32_t fused;           /* 1: the last F transform runs inside the reduction
                              (the F fields never reach device memory); 2: the
                              same in the one-pass FP32 kernel (all shells of a
                              line in one workgroup); 0: F fields in memory */
  int32_t n_terms;         /* real triple products of the expanded m-sum of eq. 41 */
  int64_t workspace_bytes; /* device memory held by the plan */
  int64_t reduce_flops;    /* floating-point operations of the reduction per
                              measurement: 2 per (output, Q row, cell) of the
                              contraction, 3 per (shell, term, cell) forming the
                              Q rows, and, when fused, 5 M log2 M per line of the
                              last F transform */
  int32_t assign_columns;  /* 1: measurements assign by columns with the z
                              transform (see tsb_options.assign_tiles) */
} tsb_plan_info;

typedef struct tsb_plan tsb_plan;

/* Validate the request and build a plan on the current device: term list
 * (3j weights), shell table, N_mode, buffers. On success *out owns device
 * memory until tsb_plan_destroy. Errors: TSB_E_ARG (NULL pointers, sizes),
 * TSB_E_UNSUPPORTED (N not 2^a 3^b, multipole outside Table 1's rules, shells
 * reaching the Nyquist frequency or r-bins reaching half the box, l > 8, a
 * grid shape the library does not cover, window multipoles in box mode,
 * shot_noise with window plans or the first- or second-vertex LOS),
 * TSB_E_NOMEM, TSB_E_DEVICE. 3PCF and window plans
 * build their separation kernels K here (one inverse transform per F slot). */
int tsb_plan_create(const tsb_grid* grid, const tsb_los* los, const tsb_kbins* bins,
                    const tsb_multipole* multipoles, int32_t n_multipoles,
                    const tsb_options* options, tsb_plan** out);

int tsb_plan_destroy(tsb_plan* plan);

/* Sizes of a plan: device bytes it holds (workspace_bytes), the number of
 * (multipole, b1, b2) entries it computes (n_pairs_total) and N_mode per bin
 * (nmode, n_bins entries, eq. 38). Any pointer may be NULL. */
int tsb_plan_query(const tsb_plan* plan, int64_t* workspace_bytes, int64_t* n_pairs_total, int64_t* nmode);

/* Host-only: validate a request exactly as tsb_plan_create does and report its
 * derived sizes (info), N_mode (nmode) and the mean |k| of each bin (k_eff),
 * without touching any device; info, nmode and k_eff may be NULL, the arrays
 * take n_bins entries. Same error codes. */
int tsb_request_query(const tsb_grid* grid, const tsb_los* los, const tsb_kbins* bins,
                      const tsb_multipole* multipoles, int32_t n_multipoles,
                      const tsb_options* options, tsb_plan_info* info, int64_t* nmode, double* k_eff);

int tsb_plan_get_info(const tsb_plan* plan, tsb_plan_info* info);

/* N_mode(b) (eq. 38) and the mean |k| of each shell, into caller-owned host
 * arrays of n_bins entries (k_eff may be NULL). */
int tsb_plan_nmode(const tsb_plan* plan, int64_t* nmode, double* k_eff);

/* The full hot path: weights, y-weighted assignment, forward FFTs, shell
 * filters, inverse FFTs, 3j-weighted reduction, normalisation.
 *   data     catalogue;
 *   randoms  catalogue, required iff box_mode == 0, else ignored;
 *   stream   hipStream_t (NULL: the default stream);
 *   B_out    host array [n_multipoles][n_bins][n_bins] (b2 fastest); entries
 *            outside the plan's pair set are NaN. TSB_BISPECTRUM: the real
 *            part of eq. 41 (eq. 52 with a global LOS), minus the shot noise
 *            of eqs. 44-46 when the plan subtracts it; TSB_3PCF: zeta of
 *            eq. 48 on r-bins; TSB_WINDOW: Q of eq. 58 (the 3PCF estimator
 *            with dn replaced by the randoms' nbar);
 *   I_out    host scalar, the normalisation I (may be NULL);
 *   alpha_out host scalar, alpha (0 in box mode) (may be NULL).
 * Synchronises the stream. Errors: TSB_E_ARG, TSB_E_INPUT (a non-finite
 * position or weight, a survey particle outside the box or at the observer,
 * or a normalisation I that is not positive, e.g. an empty catalogue, for
 * which eq. 41 is undefined), TSB_E_DEVICE. */
int tsb_measure(tsb_plan* plan, const tsb_catalog* data, const tsb_catalog* randoms,
                void* stream, double* B_out, double* I_out, double* alpha_out);

/* tsb_measure for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation. Same
 * arguments, results and errors as tsb_measure (bitwise the same B, I and
 * alpha for the same plan and catalogues), but the call allocates nothing:
 * every buffer the measurement reads and writes (grids, pass buffers, fields,
 * bucketing, partial sums, particle records, results) lives in one static
 * device array of the library, 256 MiB per device, held from the library's
 * load to the end of the process; the plan's constant tables stay with the
 * plan. The catalogues must be device memory (on_device = 1). A plan and
 * catalogue that need more than the 256 MiB fail with TSB_E_NOMEM and a
 * message giving the size they need (grids up to 64^3 with the multipoles of
 * Sec. 5.2 fit). Every call on a device shares that device's array, which
 * keeps the last call's contents (the call clears what must start at zero):
 * calls that overlap on one device race and must not be made. Synchronises
 * the stream. */
int tsb_measure_noalloc(tsb_plan* plan, const tsb_catalog* data, const tsb_catalog* randoms,
                        void* stream, double* B_out, double* I_out, double* alpha_out);

/* The shot noise S_{l1 l2 L}(k1, k2) (Sec. 4.2, eq. 44: the sum of the four
 * coincident-index terms of eq. 45 with the scalars and the w^2-weighted
 * fields of eq. 46) that the plan's last tsb_measure subtracted, into a host
 * array laid out as B_out, with the i = j != k term (the only one that
 * depends on both k1 and k2) separately in S_ijk_out (may be NULL). For 3PCF
 * plans S(r1, r2) of eq. 51, which is that term alone and zero off r1 = r2.
 * Only for plans created with shot_noise = 1 (else TSB_E_ARG). */
int tsb_plan_shot_noise(const tsb_plan* plan, double* S_out, double* S_ijk_out);

/* Stage entry point for checking the assignment: writes the y-weighted,
 * mean-subtracted density grids (before any FFT) into the caller-owned
 * device buffer grids_out, laid out [copy][channel][ix][iy][iz] with iz
 * fastest, copy = 0 (first grid) or 1 (interlaced grid, if enabled), and
 * channel c = 0..n_channels-1 in the order reported by tsb_plan_channel.
 * Element type: float (TSB_FP32) or double (TSB_FP64). Synchronises. */
int tsb_assign(tsb_plan* plan, const tsb_catalog* data, const tsb_catalog* randoms,
               void* stream, void* grids_out);

/* Which real channel c holds: y-weight of multipole L, azimuth M >= 0, and
 * part (0: Re of w y_L^M*, 1: Im of w y_L^M*). */
int tsb_plan_channel(const tsb_plan* plan, int32_t c, int32_t* L, int32_t* M, int32_t* part);

/* Stage timing. `stages` is a bit mask of stage indices (0: off, -1: every
 * stage). Every later tsb_measure records HIP events around each selected
 * stage on the caller's stream (inside the replayed graph for the graph-held
 * stages) and accumulates the elapsed times; each event pair adds a little
 * time of its own, so timing one stage perturbs a measurement less than
 * timing all. Stages (index: name): 0 weights, 1 bucket, 2 assign, 3 fwd_z, 4 fwd_y,
 * 5 fwd_x, 6 combine, 7 invF_x, 8 invF_y, 9 invF_z, 10 invG_x, 11 invG_y,
 * 12 invG_z, 13 reduce, 14 reduce_final. Each of 3..13 is one kernel launch per
 * measurement (13: one per block of 4096 outputs; when the last F transform
 * runs inside the reduction, stage 9 is empty and 13 covers both). tsb_plan_stage_times writes
 * up to n entries of accumulated milliseconds and call counts (either array may
 * be NULL) and, with reset != 0, clears the accumulators. */
int tsb_plan_set_profiling(tsb_plan* plan, int32_t stages);

/* Empirical tuning of the plan's launch schedule for the batched and
 * repeated measurements of the paper's mock campaigns (Sec. 4.4): measures
 * `data` (and `randoms` in survey mode) repeatedly on `stream`, timing each
 * candidate with HIP events over `reps` runs, and keeps the fastest (a
 * candidate replaces the default only when it is at least 2% faster)
 *   - lines per workgroup of every power-of-two FFT pass (the LDS rule, or 8,
 *     16, 32, 64 lines, at most 64 KiB of LDS);
 *   - the persistent grid of the assignment tile kernel (0.5 to 2 times its
 *     occupancy-sized default);
 *   - for the one-pass FP32 reduction, how its second phase is split: one task
 *     per (row, shell, k2), a row being one Q group or one right factor, one
 *     task per (shell, k2) covering every row, or every (slot, k2) column
 *     transformed once in LDS and then one task per (row, shell, k2);
 *   - for the unfused FP32 matrix-core reduction, its workgroup size: two of
 *     512 threads per CU (when their staged rows fit the LDS) or one of 1024.
 * These change how work is split, not the arithmetic: results stay bitwise
 * the same. The choices stay with the plan (the captured graph is rebuilt).
 * choice (may be NULL) receives 18 values: lines per workgroup per stage
 * (index as in tsb_plan_stage_times; 0 = the LDS rule), then the tile-kernel
 * workgroups, then the reduction split (1 row tasks, 0 shell tasks, 2 columns
 * then rows, -1 when the plan does not use the one-pass kernel), then the unfused reduction's
 * workgroup size (512 or 1024; -1 when the plan does not use that kernel). Clears the stage-time
 * accumulators and keeps the profiling setting. Errors as tsb_measure. */
int tsb_plan_autotune(tsb_plan* plan, const tsb_catalog* data, const tsb_catalog* randoms, void* stream,
                      int32_t reps, int32_t* choice);

/* Apply a launch schedule, e.g. one that tsb_plan_autotune returned for a
 * plan of the same request, so that a tuned schedule can be reused without
 * tuning again (serving loops, repeated campaigns). `choice` holds the 18
 * values in tsb_plan_autotune's layout: lines per workgroup per stage (0, 8,
 * 16, 32 or 64; ignored by passes whose length is not a power of two), the
 * tile-kernel workgroups (0: the occupancy default), the reduction split (1,
 * 0, 2, or -1 to leave it), the unfused reduction's workgroup size (512, 1024, or
 * -1 to leave it). Results stay bitwise the same. Errors: TSB_E_ARG. */
int tsb_plan_set_schedule(tsb_plan* plan, const int32_t* choice);
int tsb_plan_stage_times(tsb_plan* plan, int32_t n, double* ms, int64_t* calls, int32_t reset);

/* Many catalogues in one call (the batched form of eq. 41 over independent
 * mock catalogues, as in the paper's mock campaigns, Sec. 4.4). Item i measures
 * data[i] (and randoms[i] in survey mode; randoms may be NULL in box mode)
 * with plans[i] and writes B_out[i] ([n_mult][n_bins][n_bins], NaN where no
 * pair is computed), I_out[i] and alpha_out[i] (either array may be NULL).
 * Items that share a plan run one after another on that plan's own stream;
 * different plans run concurrently on their own streams, so mocks of
 * different grid sizes overlap on the device. The batch starts after the work
 * already enqueued on `stream`, later work on `stream` waits for it, and the
 * call returns when every result is on the host. Each item's result equals
 * tsb_measure on the same inputs (bitwise). Errors: as tsb_measure (first error
 * wins; results of other items are then unspecified). */
int tsb_measure_batch(tsb_plan* const* plans, const tsb_catalog* const* data,
                      const tsb_catalog* const* randoms, int32_t n, void* stream,
                      double* const* B_out, double* I_out, double* alpha_out);

/* Replay the fixed-shape part of a measurement (assignment tiles, transforms,
 * reduction) as a HIP graph captured once per plan and particle capacity
 * (default on; stage profiling always launches kernels directly). */
int tsb_plan_set_graphs(tsb_plan* plan, int32_t enable);

/* Serving: a request loop that admits measurements as they arrive.
 * tsb_server_create starts a worker thread bound to the current device that
 * runs up to max_slots measurements at once, each on its own stream and its
 * own plan workspace, and keeps the plans of recently served geometries
 * resident. Admission, oldest request first (a later request whose geometry
 * has an idle workspace may start while an earlier one waits):
 *   - an idle workspace of the request's geometry serves it, growing its
 *     particle buffers when the growth fits hbm_budget_bytes;
 *   - without room for a new workspace, a request whose geometry has a busy
 *     workspace waits for it;
 *   - otherwise idle workspaces are released, least recently used first
 *     (other geometries first), until the geometry's idle workspace can grow
 *     or a new workspace and its particle buffers fit a free slot and the
 *     budget;
 *   - a request waits only while some workspace is busy; one whose own
 *     workspace exceeds the whole budget fails with TSB_E_NOMEM.
 * Results are bitwise those of tsb_measure on the same inputs, alone or in
 * any mix.
 *   tsb_server_submit: `plan` is a template (only its request is used; it is
 *     not touched by the server and may be destroyed after the call); data /
 *     randoms point to caller-owned arrays (device or host, per on_device)
 *     that must stay valid, and B_out to caller-owned host memory that must
 *     not be read, until the request is done. Returns a ticket (> 0).
 *   tsb_server_poll: done = 1 when finished; latency_s = submit-to-finish
 *     wall time; returns the request's status (TSB_OK, or its error) once done,
 *     TSB_OK while running, TSB_E_ARG for an unknown ticket.
 *   tsb_server_wait: blocks until the ticket is done, then as poll.
 *   tsb_server_stats: the number of requests that were running on the device
 *     at the same time, at most, since the server started (peak_running), and
 *     the number of workspaces the server has released (released).
 *   tsb_server_destroy: finishes running requests, cancels queued ones
 *     (their status becomes TSB_E_CANCELLED) and frees every workspace. */
int tsb_server_create(int64_t hbm_budget_bytes, int32_t max_slots, void** server);
int tsb_server_submit(void* server, const tsb_plan* plan, const tsb_catalog* data,
                      const tsb_catalog* randoms, double* B_out, int64_t* ticket);
int tsb_server_poll(void* server, int64_t ticket, int32_t* done, double* latency_s);
int tsb_server_wait(void* server, int64_t ticket, double* latency_s);
int tsb_server_stats(void* server, int32_t* peak_running, int64_t* released);
int tsb_server_destroy(void* server);

/* ---- Masked model (Sec. 6.2), host code --------------------------------------
 * The window multipoles Q (TSB_WINDOW plans) and model three-point-function
 * multipoles zeta on the same r-bins give the masked model that the measured
 * zeta and B are compared with. Arrays are host memory, caller-owned, FP64,
 * [multipole][r1][r2] with r2 fastest. The r integrals are quadrature sums
 * sum_i w_i f(r_i) with the caller's nodes r (>= 0) and weights w. Multipoles
 * with l1, l2, L in 0..16; those with l1 + l2 + L odd contribute nothing.
 *
 * tsb_wigner_9j: the 9j symbol {l[0] l[1] l[2]; l[3] l[4] l[5]; l[6] l[7] l[8]}
 *   of App. A (eq. A5) that the coupling uses.
 * tsb_masked_zeta: eq. 63 for each output multipole (zeta_out [n_out][n_r][n_r]):
 *   sum over model (l1' l2' L') and window (l1'' l2'' L'') multipoles of
 *   N_{l1l2L} {l1'' l2'' L''; l1' l2' L'; l1 l2 L} H_{l1l2L} H_{l1 l1' l1''}
 *   H_{l2 l2' l2''} H_{L L' L''} / (H_{l1'l2'L'} H_{l1''l2''L''}) Q'' zeta',
 *   with H = 3j(. . .; 0 0 0) and N = (2l1+1)(2l2+1)(2L+1); multipoles absent from
 *   a set count as zero. With integral_constraint != 0 it also subtracts
 *   Q_{l1l2L} zeta_bar, zeta_bar of eq. 64 (the sum over multipoles in both sets
 *   of int r1^2 r2^2 Q zeta / (H^2 N), over int r1^2 r2^2 Q_000; Q_000 must be
 *   among the window multipoles), and writes zeta_bar (may be NULL; 0 without
 *   the constraint). r and w may be NULL without the constraint.
 * tsb_masked_bispectrum: eq. 68, B(k1, k2) = (-i)^{l1+l2} (4 pi)^2
 *   sum_ij w_i r_i^2 w_j r_j^2 j_l1(k1 r_i) j_l2(k2 r_j) zeta(r_i, r_j), for
 *   even l1 + l2 (real), B_out [n_k][n_k] (k2 fastest).
 * Errors: TSB_E_ARG (NULL pointers, empty sets, missing Q_000, negative r or k),
 * TSB_E_UNSUPPORTED (l outside 0..16, odd l1 + l2 in the transform), TSB_E_INPUT
 * (a vanishing integral of Q_000). */
int tsb_wigner_9j(const int32_t* l, double* out);
int tsb_masked_zeta(const tsb_multipole* model, int32_t n_model, const double* zeta,
                    const tsb_multipole* window, int32_t n_window, const double* Q,
                    const double* r, const double* w, int32_t n_r,
                    const tsb_multipole* out, int32_t n_out, int32_t integral_constraint,
                    double* zeta_out, double* zeta_bar);
int tsb_masked_bispectrum(int32_t l1, int32_t l2, const double* zeta, const double* r, const double* w,
                          int32_t n_r, const double* k, int32_t n_k, double* B_out);

const char* tsb_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TRIPOSH_H */
