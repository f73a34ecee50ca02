// Last inverse pass of the F fields (along z) fused with the 3j-weighted
// reduction (Sec. 4.2, eqs. 41-42), so the F fields never reach HBM.
//
// A workgroup owns whole z-lines (x, y fixed, M cells). For each line it
// transforms the shell slots bin group by bin group (four-step register FFT,
// one LDS transpose), turns the transformed components into
//   Q_q(x; b1) = sum_t coef_t f1_t(x; b1) g_t(x)
// and keeps the components that appear as right factors f2, then adds
// sum_x Q_q(x; b1) f2_q(x; b2) into FP64 registers, one set of outputs per
// thread. Every LDS element has a single writer per phase and partial sums
// are combined in a fixed order, so results are bitwise reproducible.
#include "fft_reg.h"
#include "tsb_internal.h"

namespace tsb {

namespace {

constexpr int kOutPerThread = 16;
constexpr int kFMaxTerms = 64, kFMaxQ = 16, kFMaxComp = 32;

// Small tables travel in the kernel arguments (scalar, uniform loads).
struct FusedTables {
  double coef[kFMaxTerms];
  int f1kind[kFMaxTerms], f1part[kFMaxTerms], g[kFMaxTerms];
  int q_t0[kFMaxQ], q_t1[kFMaxQ], q_f2row[kFMaxQ];
  int f2_kind[kFMaxComp], f2_part[kFMaxComp];   // per right-factor row
  int g_slot[kFMaxComp], g_part[kFMaxComp];     // per G component
  unsigned q_kmask[kFMaxQ];                     // slot kinds among the left factors of Q group q
};

template <typename T>
struct FusedArgs {
  typedef typename cplx<T>::type T2;
  const T2* u2;        // F slots after the x and y passes: [nf][M][M][PF]
  const int* bin_r2;   // per bin the largest |n|^2: entries beyond it were not written (zeros);
                       // null for the 3PCF, whose separation kernels fill every mode
  const T2* gfields;   // G grids [ngrid][M^3]
  const T2* tw;        // e^{-2 pi i k / M}
  int RF, PF, PFs, nb, nkinds, ngrid, ngc, nq, nf2, bpg;   // PFs: stored line stride of u2
  int ksplit;          // matrix-core contraction: cell-range splits per Q group
  const OutEntry* outs;
  int nout;
  double* partials;    // [nout][gridDim]
  FusedTables tb;
};

typedef float floatx16 __attribute__((ext_vector_type(16)));

// MF: the per-line contraction C_q(b1, b2) += sum_x Q_q(x; b1) f2_q(x; b2) runs on
// the matrix cores (FP32 32x32x2 MFMA; shells padded to 32) with one (q, cell
// range) unit per wavefront, and the line sums go to FP64 accumulators.
// UPW: matrix-core units per wavefront (two when a plan needs more than four).
template <typename T, int N1, int N2, bool MF, int UPW>
__global__ void __launch_bounds__(kBlock) fz_reduce_kernel(FusedArgs<T> a) {
  typedef typename cplx<T>::type T2;
  constexpr int M = N1 * N2;
  constexpr int LS = N2 * (N1 + 1) + 1;
  constexpr int CP = M + 1;
  const int64_t M3 = (int64_t)M * M * M;
  const int nk = a.nkinds;
  extern __shared__ char smem[];
  T* Q = (T*)smem;                                    // [nq][nb][CP]
  T* F2 = Q + (size_t)a.nq * a.nb * CP;               // [nf2][nb][CP]
  T* Gv = F2 + (size_t)a.nf2 * a.nb * CP;             // [ngc][CP]
  size_t off = ((size_t)(a.nq + a.nf2) * a.nb * CP + (size_t)a.ngc * CP) * sizeof(T);
  off = (off + 15) / 16 * 16;
  T2* stage = (T2*)(smem + off);                      // [bpg * nk][LS]
  T2* sout = stage + (size_t)a.bpg * nk * LS;         // [bpg * nk][M]
  const int tid = threadIdx.x;
  // this thread's outputs (the same for every line)
  int ob1[kOutPerThread], ob2[kOutPerThread], oq0[kOutPerThread], oq1[kOutPerThread];
  double acc[kOutPerThread];
  double acc2[UPW > 1 ? 16 : 1];   // the second unit of a wavefront
#pragma unroll
  for (int r = 0; r < (UPW > 1 ? 16 : 1); ++r) acc2[r] = 0.0;
#pragma unroll
  for (int r = 0; r < kOutPerThread; ++r) {
    acc[r] = 0.0;
    const int o = tid + r * kBlock;
    if (o < a.nout) {
      const OutEntry e = a.outs[o];
      ob1[r] = e.b1;
      ob2[r] = e.b2;
      oq0[r] = e.q0;
      oq1[r] = e.q1;
    } else {
      ob1[r] = ob2[r] = 0;
      oq0[r] = oq1[r] = 0;
    }
  }

  for (int64_t line = blockIdx.x; line < (int64_t)M * M; line += gridDim.x) {
    // G components of this line's cells
    for (int idx = tid; idx < a.ngc * M; idx += kBlock) {
      const int f = idx / M, c = idx - f * M;
      const T2 v = a.gfields[(int64_t)a.tb.g_slot[f] * M3 + line * M + c];
      Gv[(size_t)f * CP + c] = a.tb.g_part[f] ? v.y : v.x;
    }
    for (int b0 = 0; b0 < a.nb; b0 += a.bpg) {
      const int nbg = min(a.bpg, a.nb - b0);
      const int nsl = nbg * nk;
      // first half of the M-point inverse transforms of the pruned z-lines
      for (int task = tid; task < nsl * N1; task += kBlock) {
        const int sl = task / N1, n1 = task - sl * N1;
        const int64_t slot = (int64_t)b0 * nk + sl;
        const T2* src = a.u2 + (slot * M * M + line) * a.PFs;
        const int r2 = a.bin_r2 ? a.bin_r2[b0 + sl / nk] : 0x7fffffff;
        T2 v[N2];
#pragma unroll
        for (int n2 = 0; n2 < N2; ++n2) {
          int e = n1 + N1 * n2 + a.RF;
          if (e >= M) e -= M;
          T2 x;
          x.x = 0;
          x.y = 0;
          if (e < a.PF && (e - a.RF) * (e - a.RF) <= r2) x = src[e];
          v[n2] = x;
        }
        reg_fft<T, T2, N2>(v, 1);
        T2* st = stage + (size_t)sl * LS;
#pragma unroll
        for (int i = 0; i < N2; ++i) {
          const int k2 = bit_reverse<N2>(i);
          T2 w = a.tw[(n1 * k2) % M];
          w.y = -w.y;
          T2 o;
          o.x = v[i].x * w.x - v[i].y * w.y;
          o.y = v[i].x * w.y + v[i].y * w.x;
          st[k2 * (N1 + 1) + n1] = o;
        }
      }
      __syncthreads();
      // second half, natural order
      for (int task = tid; task < nsl * N2; task += kBlock) {
        const int sl = task / N2, k2 = task - sl * N2;
        const T2* st = stage + (size_t)sl * LS + k2 * (N1 + 1);
        T2 u[N1];
#pragma unroll
        for (int n1 = 0; n1 < N1; ++n1) u[n1] = st[n1];
        reg_fft<T, T2, N1>(u, 1);
        T2* so = sout + (size_t)sl * M;
#pragma unroll
        for (int i = 0; i < N1; ++i) so[k2 + N2 * bit_reverse<N1>(i)] = u[i];
      }
      __syncthreads();
      // Q rows and right-factor rows of the group's shells, one (shell, cell) per item;
      // the term loops are uniform across the workgroup
      for (int idx = tid; idx < nbg * M; idx += kBlock) {
        const int bl = idx / M, c = idx - bl * M;
        const int b = b0 + bl;
        const T2* so = sout + (size_t)bl * nk * M + c;
        for (int q = 0; q < a.nq; ++q) {
          double s = 0.0;
          for (int t = a.tb.q_t0[q]; t < a.tb.q_t1[q]; ++t) {
            const T2 v = so[(size_t)a.tb.f1kind[t] * M];
            s += a.tb.coef[t] * (double)(a.tb.f1part[t] ? v.y : v.x) * (double)Gv[(size_t)a.tb.g[t] * CP + c];
          }
          Q[((size_t)q * a.nb + b) * CP + c] = (T)s;
        }
        for (int r = 0; r < a.nf2; ++r) {
          const T2 v = so[(size_t)a.tb.f2_kind[r] * M];
          F2[((size_t)r * a.nb + b) * CP + c] = a.tb.f2_part[r] ? v.y : v.x;
        }
      }
      __syncthreads();
    }
    if constexpr (MF) {
      const int wave = tid >> 6, lane = tid & 63;
#pragma unroll
      for (int uu = 0; uu < UPW; ++uu) {
        const int unit = wave + uu * (kBlock / 64);
        if (unit < a.nq * a.ksplit) {
          const int q = unit / a.ksplit, sp = unit - q * a.ksplit;
          const int b = lane & 31, kh = lane >> 5;
          const bool live = b < a.nb;
          const T* qr = Q + ((size_t)q * a.nb + (live ? b : 0)) * CP + kh;
          const T* fr = F2 + ((size_t)a.tb.q_f2row[q] * a.nb + (live ? b : 0)) * CP + kh;
          const int kl = M / a.ksplit, k0 = sp * kl;   // kl is even
          floatx16 c = {};
          for (int kk = k0; kk < k0 + kl; kk += 2) {
            const float av = live ? (float)qr[kk] : 0.f;
            const float bv = live ? (float)fr[kk] : 0.f;
            c = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, c, 0, 0, 0);
          }
          if (uu == 0) {
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[r] += (double)c[r];
          } else {
#pragma unroll
            for (int r = 0; r < (UPW > 1 ? 16 : 1); ++r) acc2[r] += (double)c[r];
          }
        }
      }
    } else {
      // sum over the line's cells for every output of this thread
#pragma unroll
      for (int r = 0; r < kOutPerThread; ++r) {
        if (tid + r * kBlock >= a.nout) break;
        double s = 0.0;
        for (int q = oq0[r]; q < oq1[r]; ++q) {
          const T* qr = Q + ((size_t)q * a.nb + ob1[r]) * CP;
          const T* fr = F2 + ((size_t)a.tb.q_f2row[q] * a.nb + ob2[r]) * CP;
          for (int c = 0; c < M; ++c) s += (double)qr[c] * (double)fr[c];
        }
        acc[r] += s;
      }
    }
    __syncthreads();
  }
  if constexpr (MF) {
    // unit tiles to LDS (row i = 8 (r / 4) + 4 (lane / 32) + r % 4, column lane % 32),
    // then each output sums its Q groups and cell ranges in a fixed order
    double* Ct = (double*)smem;   // [units][32][32]
    const int wave = tid >> 6, lane = tid & 63;
#pragma unroll
    for (int uu = 0; uu < UPW; ++uu) {
      const int unit = wave + uu * (kBlock / 64);
      if (unit < a.nq * a.ksplit) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int i = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3), j = lane & 31;
          Ct[((size_t)unit * 32 + i) * 32 + j] = uu == 0 ? acc[r] : acc2[UPW > 1 ? r : 0];
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kOutPerThread; ++r) {
      const int o = tid + r * kBlock;
      if (o >= a.nout) break;
      double v = 0.0;
      for (int q = oq0[r]; q < oq1[r]; ++q)
        for (int sp = 0; sp < a.ksplit; ++sp) v += Ct[((size_t)(q * a.ksplit + sp) * 32 + ob1[r]) * 32 + ob2[r]];
      a.partials[(size_t)o * gridDim.x + blockIdx.x] = v;
    }
  } else {
#pragma unroll
    for (int r = 0; r < kOutPerThread; ++r) {
      const int o = tid + r * kBlock;
      if (o < a.nout) a.partials[(size_t)o * gridDim.x + blockIdx.x] = acc[r];
    }
  }
}

// ---------------------------------------------------------------------------
// FP32 plans, the shells of a line in one or two groups: 512 threads, two
// barriers per group.
//   phase 1: first-level transforms of every (slot, n1) of the group, inputs
//            prefetched into registers while the previous group finishes;
//   phase 2: per (shell, k2) the second-level transforms of the slot kinds
//            (all together when a shell has at most four, else one at a time),
//            turned straight into the Q rows and right-factor rows of N1
//            cells;
//   then, once every shell of the line is done, the contraction on the matrix
//   cores (units of (q, cell range) over the eight wavefronts), which overlaps
//   the next line's loads and first phase.

constexpr int kWBlock = 512;
constexpr int kWOut = 8;       // outputs per thread
constexpr int kWGPre = 2;      // G values per thread and line
constexpr int kWGroups = 256;  // workgroups of the one-pass kernel
constexpr int kWMaxQ = 8;      // Q groups
constexpr size_t kLdsPerCU = 160 * 1024;   // gfx950: the whole LDS of a CU for one workgroup

// sq[i] += cf * part(row[i]) * g(c_i) for the N1 cells c_i = k2 + N2 bitrev(i)
template <int N1, int N2>
__device__ inline void add_term(float (&sq)[N1], const float2 (&row)[N1], int part, float cf, const float* gr) {
#pragma unroll
  for (int i = 0; i < N1; ++i) {
    const float f = part ? row[i].y : row[i].x;
    sq[i] += cf * f * gr[N2 * bit_reverse<N1>(i)];
  }
}

template <int N1, int N2>
__device__ inline void put_row(float* frow, const float2 (&row)[N1], int part) {
#pragma unroll
  for (int i = 0; i < N1; ++i) frow[N2 * bit_reverse<N1>(i)] = part ? row[i].y : row[i].x;
}

// The same from a row already transformed in LDS (entry i holds cell c_i).
template <int N1, int N2>
__device__ inline void add_term_lds(float (&sq)[N1], const float2* row, int part, float cf, const float* gr) {
#pragma unroll
  for (int i = 0; i < N1; ++i) {
    const float2 v = row[i];
    const float f = part ? v.y : v.x;
    sq[i] += cf * f * gr[N2 * bit_reverse<N1>(i)];
  }
}

template <int N1, int N2>
__device__ inline void put_row(float* frow, const float (&row)[N1]) {
#pragma unroll
  for (int i = 0; i < N1; ++i) frow[N2 * bit_reverse<N1>(i)] = row[i];
}

constexpr int kWKinds = 4;     // slot kinds per shell held in registers at once (KR mode)

// KR: the slot kinds of a shell (at most kWKinds) are transformed together and
// held in registers while the Q rows are formed one group at a time;
// otherwise the kinds are transformed one at a time and the Q rows of up to
// NQ groups (2, 4 or 8) are held in registers. GR: the shells of a line come
// in more than one group. RT: the second phase runs one task per (row, shell,
// k2), a row being a Q group or a right factor, so that small shell groups
// still fill the workgroup; each task transforms the kinds its row needs.
// The terms of a row are added in the same order as without RT (term order
// with KR, kind by kind without), so RT changes only the split of the work.
// KT: the second phase first transforms every (slot, k2) column once, in
// place in LDS, then forms the rows from the transformed columns (no
// transform repeated per row; the same term order as KR for at most kWKinds
// kinds, kind by kind beyond, so KT too changes only the split of the work).
template <int N1, int N2, int NQ, bool KR, bool GR, bool RT, bool KT = false>
__global__ void __launch_bounds__(kWBlock) fz_reduce_wide_kernel(FusedArgs<float> a) {
  typedef float2 T2;
  constexpr int M = N1 * N2;
  constexpr int LS = N2 * (N1 + 1) + 1;
  constexpr int CP = M + 1;
  const int64_t M3 = (int64_t)M * M * M, lines = (int64_t)M * M;
  const int nk = a.nkinds, nb = a.nb, nq = a.nq, bpg = GR ? a.bpg : nb;
  const int ngrp = GR ? (nb + bpg - 1) / bpg : 1;
  extern __shared__ char smem[];
  float* Q = (float*)smem;                         // [nq][nb][CP]
  float* F2 = Q + (size_t)nq * nb * CP;            // [nf2][nb][CP]
  float* Gv = F2 + (size_t)a.nf2 * nb * CP;        // [ngc][CP]
  size_t off = ((size_t)(nq + a.nf2) * nb * CP + (size_t)a.ngc * CP) * sizeof(float);
  off = (off + 15) / 16 * 16;
  T2* tw = (T2*)(smem + off);                      // [M] e^{+2 pi i k / M}
  T2* stage = tw + M;                              // [bpg * nk][LS]
  const int tid = threadIdx.x;
  for (int k = tid; k < M; k += kWBlock) {
    T2 w = a.tw[k];
    w.y = -w.y;
    tw[k] = w;
  }
  const int wave = tid >> 6, lane = tid & 63;
  const int nunits = nq * a.ksplit;
  double acc[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0;
  // phase-1 task of this thread in a group (slot sl of the group, n1) and its
  // prefetched inputs
  const int sl = tid / N1, n1 = tid - (tid / N1) * N1;
  T2 pv[N2];
  float gpre[kWGPre];
  auto group_slots = [&](int g) { return min(bpg, nb - g * bpg) * nk; };
  auto prefetch = [&](int64_t line, int g) {
    if (sl < group_slots(g)) {
      const T2* src = a.u2 + ((int64_t)(g * bpg * nk + sl) * M * M + line) * a.PFs;
      const int r2 = a.bin_r2 ? a.bin_r2[g * bpg + sl / nk] : 0x7fffffff;
#pragma unroll
      for (int n2 = 0; n2 < N2; ++n2) {
        int e = n1 + N1 * n2 + a.RF;
        if (e >= M) e -= M;
        T2 x;
        x.x = 0.f;
        x.y = 0.f;
        if (e < a.PF && (e - a.RF) * (e - a.RF) <= r2) x = src[e];
        pv[n2] = x;
      }
    }
    if (g == 0) {
#pragma unroll
      for (int j = 0; j < kWGPre; ++j) {
        const int idx = tid + j * kWBlock;
        gpre[j] = 0.f;
        if (idx < a.ngc * M) {
          const int f = idx / M, c = idx - f * M;
          const T2 v = a.gfields[(int64_t)a.tb.g_slot[f] * M3 + line * M + c];
          gpre[j] = a.tb.g_part[f] ? v.y : v.x;
        }
      }
    }
  };
  int64_t line = blockIdx.x;
  if (line < lines) prefetch(line, 0);
  __syncthreads();   // twiddles
  for (; line < lines; line += gridDim.x) {
#pragma unroll
    for (int j = 0; j < kWGPre; ++j) {
      const int idx = tid + j * kWBlock;
      if (idx < a.ngc * M) {
        const int f = idx / M, c = idx - f * M;
        Gv[(size_t)f * CP + c] = gpre[j];
      }
    }
    for (int g = 0; g < ngrp; ++g) {
      const int b0 = g * bpg, nbg = min(bpg, nb - b0);
      if (sl < nbg * nk) {
        reg_fft<float, T2, N2>(pv, 1);
        T2* st = stage + (size_t)sl * LS;
#pragma unroll
        for (int i = 0; i < N2; ++i) {
          const int k2 = bit_reverse<N2>(i);
          const T2 w = tw[(n1 * k2) % M];
          T2 o;
          o.x = pv[i].x * w.x - pv[i].y * w.y;
          o.y = pv[i].x * w.y + pv[i].y * w.x;
          st[k2 * (N1 + 1) + n1] = o;
        }
      }
      __syncthreads();
      if (g + 1 < ngrp) prefetch(line, g + 1);
      else if (line + gridDim.x < lines) prefetch(line + gridDim.x, 0);
      if constexpr (KT) {
      // second-level transforms of every (slot, k2) column, in place
      for (int task = tid; task < nbg * nk * N2; task += kWBlock) {
        const int sk = task / N2, k2 = task - sk * N2;
        T2* st = stage + (size_t)sk * LS + k2 * (N1 + 1);
        T2 u[N1];
#pragma unroll
        for (int j = 0; j < N1; ++j) u[j] = st[j];
        reg_fft<float, T2, N1>(u, 1);
#pragma unroll
        for (int j = 0; j < N1; ++j) st[j] = u[j];
      }
      __syncthreads();
      const int per_row = nbg * N2, nrow = nq + a.nf2;
      const bool korder = nk <= kWKinds;
      for (int task = tid; task < nrow * per_row; task += kWBlock) {
        const int r = task / per_row, rest = task - r * per_row;
        const int bl = rest / N2, k2 = rest - bl * N2, b = b0 + bl;
        const T2* col = stage + (size_t)(bl * nk) * LS + k2 * (N1 + 1);   // kind k at col + k LS
        if (r < nq) {
          float sq[N1];
#pragma unroll
          for (int i = 0; i < N1; ++i) sq[i] = 0.f;
          if (korder) {
            for (int t = a.tb.q_t0[r]; t < a.tb.q_t1[r]; ++t)
              add_term_lds<N1, N2>(sq, col + (size_t)a.tb.f1kind[t] * LS, a.tb.f1part[t], (float)a.tb.coef[t],
                                   Gv + (size_t)a.tb.g[t] * CP + k2);
          } else {
            const unsigned kmask = a.tb.q_kmask[r];
            for (int k = 0; k < nk; ++k) {
              if (!((kmask >> k) & 1u)) continue;
              for (int t = a.tb.q_t0[r]; t < a.tb.q_t1[r]; ++t) {
                if (a.tb.f1kind[t] != k) continue;
                add_term_lds<N1, N2>(sq, col + (size_t)k * LS, a.tb.f1part[t], (float)a.tb.coef[t],
                                     Gv + (size_t)a.tb.g[t] * CP + k2);
              }
            }
          }
          put_row<N1, N2>(Q + ((size_t)r * nb + b) * CP + k2, sq);
        } else {
          const int rr = r - nq;
          const T2* src = col + (size_t)a.tb.f2_kind[rr] * LS;
          T2 u[N1];
#pragma unroll
          for (int j = 0; j < N1; ++j) u[j] = src[j];
          put_row<N1, N2>(F2 + ((size_t)rr * nb + b) * CP + k2, u, a.tb.f2_part[rr]);
        }
      }
      } else if constexpr (RT) {
      const int per_row = nbg * N2, nrow = nq + a.nf2;
      for (int task = tid; task < nrow * per_row; task += kWBlock) {
        const int r = task / per_row, rest = task - r * per_row;
        const int bl = rest / N2, k2 = rest - bl * N2, b = b0 + bl;
        auto load_kind = [&](int k, T2 (&u)[N1]) {
          const T2* st = stage + (size_t)(bl * nk + k) * LS + k2 * (N1 + 1);
#pragma unroll
          for (int j = 0; j < N1; ++j) u[j] = st[j];
          reg_fft<float, T2, N1>(u, 1);
        };
        if (r < nq) {
          float sq[N1];
#pragma unroll
          for (int i = 0; i < N1; ++i) sq[i] = 0.f;
          const unsigned kmask = a.tb.q_kmask[r];
          if constexpr (KR) {
            // every kind the row needs in registers, then the terms in order
            T2 u[kWKinds][N1];
#pragma unroll
            for (int k = 0; k < kWKinds; ++k) {
              if (k < nk && ((kmask >> k) & 1u)) {
                load_kind(k, u[k]);
              } else {
#pragma unroll
                for (int j = 0; j < N1; ++j) u[k][j] = make_float2(0.f, 0.f);
              }
            }
            for (int t = a.tb.q_t0[r]; t < a.tb.q_t1[r]; ++t) {
              const float cf = (float)a.tb.coef[t];
              const int part = a.tb.f1part[t];
              const float* gr = Gv + (size_t)a.tb.g[t] * CP + k2;
              switch (a.tb.f1kind[t]) {
                case 0: add_term<N1, N2>(sq, u[0], part, cf, gr); break;
                case 1: add_term<N1, N2>(sq, u[1], part, cf, gr); break;
                case 2: add_term<N1, N2>(sq, u[2], part, cf, gr); break;
                default: add_term<N1, N2>(sq, u[3], part, cf, gr); break;
              }
            }
          } else {
            for (int k = 0; k < nk; ++k) {
              if (!((kmask >> k) & 1u)) continue;
              T2 u[N1];
              load_kind(k, u);
              for (int t = a.tb.q_t0[r]; t < a.tb.q_t1[r]; ++t) {
                if (a.tb.f1kind[t] != k) continue;
                add_term<N1, N2>(sq, u, a.tb.f1part[t], (float)a.tb.coef[t], Gv + (size_t)a.tb.g[t] * CP + k2);
              }
            }
          }
          put_row<N1, N2>(Q + ((size_t)r * nb + b) * CP + k2, sq);
        } else {
          const int rr = r - nq;
          T2 u[N1];
          load_kind(a.tb.f2_kind[rr], u);
          put_row<N1, N2>(F2 + ((size_t)rr * nb + b) * CP + k2, u, a.tb.f2_part[rr]);
        }
      }
      } else if constexpr (KR) {
      for (int task = tid; task < nbg * N2; task += kWBlock) {
        const int bl = task / N2, k2 = task - bl * N2, b = b0 + bl;
        T2 u[kWKinds][N1];
#pragma unroll
        for (int k = 0; k < kWKinds; ++k) {
          if (k < nk) {
            const T2* st = stage + (size_t)(bl * nk + k) * LS + k2 * (N1 + 1);
#pragma unroll
            for (int j = 0; j < N1; ++j) u[k][j] = st[j];
            reg_fft<float, T2, N1>(u[k], 1);
          } else {
#pragma unroll
            for (int j = 0; j < N1; ++j) u[k][j] = make_float2(0.f, 0.f);
          }
        }
        // rows of the N1 cells c_i = k2 + N2 bitrev(i); slot kinds are picked by
        // uniform branches so that every register index stays static
        for (int q = 0; q < nq; ++q) {
          float sq[N1];
#pragma unroll
          for (int i = 0; i < N1; ++i) sq[i] = 0.f;
          for (int t = a.tb.q_t0[q]; t < a.tb.q_t1[q]; ++t) {
            const float cf = (float)a.tb.coef[t];
            const int part = a.tb.f1part[t];
            const float* gr = Gv + (size_t)a.tb.g[t] * CP + k2;
            switch (a.tb.f1kind[t]) {
              case 0: add_term<N1, N2>(sq, u[0], part, cf, gr); break;
              case 1: add_term<N1, N2>(sq, u[1], part, cf, gr); break;
              case 2: add_term<N1, N2>(sq, u[2], part, cf, gr); break;
              default: add_term<N1, N2>(sq, u[3], part, cf, gr); break;
            }
          }
          put_row<N1, N2>(Q + ((size_t)q * nb + b) * CP + k2, sq);
        }
        for (int r = 0; r < a.nf2; ++r) {
          float* frow = F2 + ((size_t)r * nb + b) * CP + k2;
          const int part = a.tb.f2_part[r];
          switch (a.tb.f2_kind[r]) {
            case 0: put_row<N1, N2>(frow, u[0], part); break;
            case 1: put_row<N1, N2>(frow, u[1], part); break;
            case 2: put_row<N1, N2>(frow, u[2], part); break;
            default: put_row<N1, N2>(frow, u[3], part); break;
          }
        }
      }
      } else {
      for (int task = tid; task < nbg * N2; task += kWBlock) {
        const int bl = task / N2, k2 = task - bl * N2, b = b0 + bl;
        float sq[NQ][N1];
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
          for (int i = 0; i < N1; ++i) sq[q][i] = 0.f;
        for (int k = 0; k < nk; ++k) {
          // kind k of shell b: second-level transform of cells c_i = k2 + N2 bitrev(i)
          T2 u[N1];
          const T2* st = stage + (size_t)(bl * nk + k) * LS + k2 * (N1 + 1);
#pragma unroll
          for (int j = 0; j < N1; ++j) u[j] = st[j];
          reg_fft<float, T2, N1>(u, 1);
          // its terms of each Q row (uniform branches keep register indices static)
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            if (q >= nq) break;
            for (int t = a.tb.q_t0[q]; t < a.tb.q_t1[q]; ++t) {
              if (a.tb.f1kind[t] != k) continue;
              add_term<N1, N2>(sq[q], u, a.tb.f1part[t], (float)a.tb.coef[t], Gv + (size_t)a.tb.g[t] * CP + k2);
            }
          }
          for (int r = 0; r < a.nf2; ++r)
            if (a.tb.f2_kind[r] == k) put_row<N1, N2>(F2 + ((size_t)r * nb + b) * CP + k2, u, a.tb.f2_part[r]);
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          if (q >= nq) break;
          put_row<N1, N2>(Q + ((size_t)q * nb + b) * CP + k2, sq[q]);
        }
      }
      }
      __syncthreads();
    }
    if (wave < nunits) {
      const int q = wave / a.ksplit, sp = wave - q * a.ksplit;
      const int b = lane & 31, kh = lane >> 5;
      const bool live = b < nb;
      const float* qr = Q + ((size_t)q * nb + (live ? b : 0)) * CP + kh;
      const float* fr = F2 + ((size_t)a.tb.q_f2row[q] * nb + (live ? b : 0)) * CP + kh;
      const int kl = M / a.ksplit, k0 = sp * kl;   // kl is a multiple of 8
      floatx16 c = {};
      for (int kk = k0; kk < k0 + kl; kk += 8) {
        // four steps' operands first, so that one LDS wait covers four MFMAs
        float av[4], bv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          av[j] = live ? qr[kk + 2 * j] : 0.f;
          bv[j] = live ? fr[kk + 2 * j] : 0.f;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) c = __builtin_amdgcn_mfma_f32_32x32x2f32(av[j], bv[j], c, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[r] += (double)c[r];
    }
  }
  __syncthreads();
  double* Ct = (double*)smem;   // [units][32][32]
  if (wave < nunits) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3), j = lane & 31;
      Ct[((size_t)wave * 32 + i) * 32 + j] = acc[r];
    }
  }
  __syncthreads();
  for (int o = tid; o < a.nout; o += kWBlock) {
    const OutEntry e = a.outs[o];
    double v = 0.0;
    for (int q = e.q0; q < e.q1; ++q)
      for (int sp = 0; sp < a.ksplit; ++sp) v += Ct[((size_t)(q * a.ksplit + sp) * 32 + e.b1) * 32 + e.b2];
    a.partials[(size_t)o * gridDim.x + blockIdx.x] = v;
  }
}

// Shells per group of the one-pass kernel at the given group size.
size_t wide_lds_bytes(const Plan& P, int bpg) {
  const int M = P.M;
  const int N2 = M >= 128 ? 16 : 8;
  const int N1 = M / N2;
  const size_t LS = (size_t)N2 * (N1 + 1) + 1;
  size_t off = ((P.qgroups.size() + P.nf2) * P.nb + P.gcomp.size()) * (size_t)(M + 1) * sizeof(float);
  off = (off + 15) / 16 * 16;
  const size_t need = off + (size_t)M * 8 + (size_t)bpg * P.fkinds.size() * LS * 8;
  const size_t units = P.qgroups.size() * (size_t)std::max<size_t>(1, 8 / P.qgroups.size());
  const size_t tiles = units * 32 * 32 * sizeof(double);
  return need > tiles ? need : tiles;
}

// Shells per group for the one-pass FP32 kernel (the fewest groups whose
// first-phase tasks fit the workgroup and whose LDS fits), or 0 when the
// kernel does not apply (shape limits of its register and LDS layout).
int wide_group(const Plan& P) {
  if (P.precision != TSB_FP32) return 0;
  if (!(P.M == 64 || P.M == 128)) return 0;   // N1 = 8
  const int N2 = P.M >= 128 ? 16 : 8, N1 = P.M / N2;
  const int nq = (int)P.qgroups.size(), nk = (int)P.fkinds.size();
  if (P.nb > 32 || nq < 1 || nq > kWMaxQ || nk < 1) return 0;
  if ((int)P.gcomp.size() * P.M > kWGPre * kWBlock) return 0;
  if ((int)P.outs.size() > kWOut * kWBlock) return 0;
  if ((int)P.terms.size() > kFMaxTerms || P.nf2 > kFMaxComp || (int)P.gcomp.size() > kFMaxComp) return 0;
  for (int ng = 1; ng <= 4; ++ng) {
    const int bpg = (P.nb + ng - 1) / ng;
    if (bpg * nk * N1 > kWBlock) continue;
    if (wide_lds_bytes(P, bpg) <= kLdsPerCU) return bpg;
  }
  return 0;
}

// Matrix-core contraction (FP32 plans, up to 32 shells and 4 Q groups): cell
// splits per Q group so that the units fill the four wavefronts.
int fused_ksplit(const Plan& P) {
  const int nq = (int)P.qgroups.size();
  if (P.precision != TSB_FP32 || P.nb > 32 || nq < 1 || nq > 8 || P.M % 2 != 0) return 0;
  // up to eight (Q group, cell range) units, two per wavefront of the
  // 256-thread kernel; every cell range an even number of cells
  int ks = std::max(1, 8 / nq);
  while (ks > 1 && P.M % (2 * ks) != 0) ks /= 2;
  return ks;
}

int fused_units(const Plan& P) { return (int)P.qgroups.size() * fused_ksplit(P); }

template <typename T>
size_t fused_lds_bytes(const Plan& P, int bpg) {
  typedef typename cplx<T>::type T2;
  const int M = P.M;
  const int N2 = M >= 128 ? 16 : (M >= 32 ? 8 : 4);
  const int N1 = M / N2;
  const size_t LS = (size_t)N2 * (N1 + 1) + 1;
  size_t off = ((P.qgroups.size() + P.nf2) * P.nb + P.gcomp.size()) * (size_t)(M + 1) * sizeof(T);
  off = (off + 15) / 16 * 16;
  const size_t need = off + (size_t)bpg * P.fkinds.size() * (LS + M) * sizeof(T2);
  const size_t tiles = (size_t)fused_units(P) * 32 * 32 * sizeof(double);
  return need > tiles ? need : tiles;
}

template <typename T, int N1, int N2>
int fused_launch(Plan& P, hipStream_t s) {
  typedef typename cplx<T>::type T2;
  FusedArgs<T> a{};
  a.u2 = (const T2*)P.d_u2;
  a.bin_r2 = P.d_kslot ? nullptr : P.d_bin_r2;   // separation kernels fill every mode
  a.gfields = (const T2*)P.d_fields + P.g_offset;
  a.tw = (const T2*)P.d_tw_m;
  a.RF = P.RF;
  a.PF = P.PF;
  a.PFs = (int)pad_line(P.PF);
  a.nb = P.nb;
  a.nkinds = (int)P.fkinds.size();
  a.ngrid = (int)P.grids.size();
  a.ngc = (int)P.gcomp.size();
  a.nq = (int)P.qgroups.size();
  a.nf2 = P.nf2;
  a.bpg = P.fused_bpg;
  a.outs = P.d_outs;
  a.nout = (int)P.outs.size();
  a.partials = P.d_partials;
  for (size_t t = 0; t < P.terms.size(); ++t) {
    a.tb.coef[t] = P.terms[t].coef;
    a.tb.f1kind[t] = P.fcomp[P.terms[t].f1].slot;
    a.tb.f1part[t] = P.fcomp[P.terms[t].f1].part;
    a.tb.g[t] = P.terms[t].g;
  }
  for (size_t q = 0; q < P.qgroups.size(); ++q) {
    a.tb.q_t0[q] = P.qgroups[q].t0;
    a.tb.q_t1[q] = P.qgroups[q].t1;
    a.tb.q_f2row[q] = P.f2idx[P.qgroups[q].f2];
  }
  for (size_t f = 0; f < P.fcomp.size(); ++f)
    if (P.f2idx[f] >= 0) {
      a.tb.f2_kind[P.f2idx[f]] = P.fcomp[f].slot;
      a.tb.f2_part[P.f2idx[f]] = P.fcomp[f].part;
    }
  for (size_t f = 0; f < P.gcomp.size(); ++f) {
    a.tb.g_slot[f] = P.gcomp[f].slot;
    a.tb.g_part[f] = P.gcomp[f].part;
  }
  for (size_t q = 0; q < P.qgroups.size(); ++q) {
    a.tb.q_kmask[q] = 0u;
    for (int t = P.qgroups[q].t0; t < P.qgroups[q].t1; ++t) a.tb.q_kmask[q] |= 1u << a.tb.f1kind[t];
  }
  const size_t lds = fused_lds_bytes<T>(P, P.fused_bpg);
  prof_begin(P, kStReduce, s);
  if (P.fused_wide) {
    a.ksplit = std::max(1, 8 / a.nq);
    if constexpr (std::is_same<T, float>::value && N1 == 8 && N1 * N2 >= 64) {
      const size_t wl = wide_lds_bytes(P, P.fused_bpg);
      const bool grouped = P.fused_bpg < P.nb;
      const dim3 grid(P.red_wg), block(kWBlock);
      if (P.fused_rt == 2 && !grouped)
        hipLaunchKernelGGL((fz_reduce_wide_kernel<N1, N2, 1, false, false, false, true>), grid, block, wl, s, a);
      else if (P.fused_rt == 2)
        hipLaunchKernelGGL((fz_reduce_wide_kernel<N1, N2, 1, false, true, false, true>), grid, block, wl, s, a);
      else if (P.fused_rt && a.nkinds <= kWKinds && !grouped)
        hipLaunchKernelGGL((fz_reduce_wide_kernel<N1, N2, 1, true, false, true>), grid, block, wl, s, a);
      else if (P.fused_rt && a.nkinds <= kWKinds)
        hipLaunchKernelGGL((fz_reduce_wide_kernel<N1, N2, 1, true, true, true>), grid, block, wl, s, a);
      else if (P.fused_rt)
        hipLaunchKernelGGL((fz_reduce_wide_kernel<N1, N2, 1, false, true, true>), grid, block, wl, s, a);
      else if (a.nkinds <= kWKinds && !grouped)
        hipLaunchKernelGGL((fz_reduce_wide_kernel<N1, N2, 1, true, false, false>), grid, block, wl, s, a);
      else if (a.nkinds <= kWKinds)
        hipLaunchKernelGGL((fz_reduce_wide_kernel<N1, N2, 1, true, true, false>), grid, block, wl, s, a);
      else if (a.nq <= 2)
        hipLaunchKernelGGL((fz_reduce_wide_kernel<N1, N2, 2, false, true, false>), grid, block, wl, s, a);
      else if (a.nq <= 4)
        hipLaunchKernelGGL((fz_reduce_wide_kernel<N1, N2, 4, false, true, false>), grid, block, wl, s, a);
      else
        hipLaunchKernelGGL((fz_reduce_wide_kernel<N1, N2, 8, false, true, false>), grid, block, wl, s, a);
      prof_end(P, kStReduce, s);
      TSB_HIP(hipGetLastError());
      return TSB_OK;
    }
    return fail(TSB_E_UNSUPPORTED, "fused reduction: one-pass kernel does not cover this shape");
  }
  a.ksplit = fused_ksplit(P);
  if (a.ksplit > 0 && a.nq * a.ksplit > kBlock / 64)
    hipLaunchKernelGGL((fz_reduce_kernel<T, N1, N2, true, 2>), dim3(P.red_wg), dim3(kBlock), lds, s, a);
  else if (a.ksplit > 0)
    hipLaunchKernelGGL((fz_reduce_kernel<T, N1, N2, true, 1>), dim3(P.red_wg), dim3(kBlock), lds, s, a);
  else
    hipLaunchKernelGGL((fz_reduce_kernel<T, N1, N2, false, 1>), dim3(P.red_wg), dim3(kBlock), lds, s, a);
  prof_end(P, kStReduce, s);
  TSB_HIP(hipGetLastError());
  return TSB_OK;
}

template <typename T>
int fused_impl(Plan& P, hipStream_t s) {
  switch (P.M) {
    case 16: return fused_launch<T, 4, 4>(P, s);
    case 32: return fused_launch<T, 4, 8>(P, s);
    case 64: return fused_launch<T, 8, 8>(P, s);
    case 128: return fused_launch<T, 8, 16>(P, s);
    case 256: return fused_launch<T, 16, 16>(P, s);
    default: return fail(TSB_E_UNSUPPORTED, "fused reduction: unsupported M");
  }
}

}  // namespace

// Planning: whether the fused path applies and its bin-group size.
void plan_fused(Plan& P) {
  P.fused = false;
  if (P.unfused == 1) return;
  const int M = P.M;
  if (!(M == 16 || M == 32 || M == 64 || M == 128 || M == 256)) return;
  if ((int)P.outs.size() > kOutPerThread * kBlock || P.outs.empty()) return;
  if ((int)P.terms.size() > kFMaxTerms || (int)P.qgroups.size() > kFMaxQ || P.nf2 > kFMaxComp ||
      (int)P.gcomp.size() > kFMaxComp)
    return;
  const int wide_bpg = wide_group(P);
  P.fused_wide = wide_bpg > 0;
  // Shells in groups make the one-pass kernel re-stage every line per group;
  // when the F fields are affordable the unfused matrix-core reduction is
  // faster (the 128^3 box with {000, 110, 202, 112}: 1.84 against 2.14 ms)
  const int64_t f_bytes = (int64_t)P.nb * (int64_t)P.fkinds.size() * M * M * M * 8;
  if (P.unfused == 0 && P.fused_wide && wide_bpg < P.nb && unfused_mfma_applies(P) && f_bytes <= (4LL << 30)) {
    P.fused_wide = false;
    return;
  }
  if (P.fused_wide) {
    // one workgroup of 512 threads per compute unit (its LDS fills one): 256 on MI355X
    P.fused = true;
    P.fused_bpg = wide_bpg;
    P.red_wg = std::min<int>(kWGroups, M * M);
    return;
  }
  const bool f64 = P.precision == TSB_FP64;
  for (int bpg = P.nb; bpg >= 1; --bpg) {
    const size_t b = f64 ? fused_lds_bytes<double>(P, bpg) : fused_lds_bytes<float>(P, bpg);
    if (b <= 76 * 1024 || (bpg == 1 && b <= 150 * 1024)) {
      P.fused = true;
      P.fused_bpg = bpg;
      return;
    }
  }
}

int run_fused(Plan& P, hipStream_t s) {
  return P.precision == TSB_FP64 ? fused_impl<double>(P, s) : fused_impl<float>(P, s);
}

}  // namespace tsb
