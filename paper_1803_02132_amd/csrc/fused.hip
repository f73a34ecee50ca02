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
};

template <typename T>
struct FusedArgs {
  typedef typename cplx<T>::type T2;
  const T2* u2;        // F slots after the x and y passes: [nf][M][M][PF]
  const T2* gfields;   // G grids [ngrid][M^3]
  const T2* tw;        // e^{-2 pi i k / M}
  int RF, PF, nb, nkinds, ngrid, ngc, nq, nf2, bpg;
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
template <typename T, int N1, int N2, bool MF>
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
        const T2* src = a.u2 + (slot * M * M + line) * a.PF;
        T2 v[N2];
#pragma unroll
        for (int n2 = 0; n2 < N2; ++n2) {
          int e = n1 + N1 * n2 + a.RF;
          if (e >= M) e -= M;
          T2 x;
          x.x = 0;
          x.y = 0;
          if (e < a.PF) x = src[e];
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
      if (wave < a.nq * a.ksplit) {
        const int q = wave / a.ksplit, sp = wave - q * a.ksplit;
        const int b = lane & 31, kh = lane >> 5;
        const bool live = b < a.nb;
        const T* qr = Q + ((size_t)q * a.nb + (live ? b : 0)) * CP + kh;
        const T* fr = F2 + ((size_t)a.tb.q_f2row[q] * a.nb + (live ? b : 0)) * CP + kh;
        const int kl = M / a.ksplit, k0 = sp * kl;
        floatx16 c = {};
        for (int kk = k0; kk < k0 + kl; kk += 2) {
          const float av = live ? (float)qr[kk] : 0.f;
          const float bv = live ? (float)fr[kk] : 0.f;
          c = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, c, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] += (double)c[r];
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
    if (wave < a.nq * a.ksplit) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3), j = lane & 31;
        Ct[((size_t)wave * 32 + i) * 32 + j] = acc[r];
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

// Matrix-core contraction (FP32 plans, up to 32 shells and 4 Q groups): cell
// splits per Q group so that the units fill the four wavefronts.
int fused_ksplit(const Plan& P) {
  const int nq = (int)P.qgroups.size();
  if (P.precision != TSB_FP32 || P.nb > 32 || nq < 1 || nq > 4) return 0;
  return nq == 1 ? 4 : (nq == 2 ? 2 : 1);
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
  a.gfields = (const T2*)P.d_fields + P.g_offset;
  a.tw = (const T2*)P.d_tw_m;
  a.RF = P.RF;
  a.PF = P.PF;
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
  const size_t lds = fused_lds_bytes<T>(P, P.fused_bpg);
  prof_begin(P, kStReduce, s);
  a.ksplit = fused_ksplit(P);
  if (a.ksplit > 0)
    hipLaunchKernelGGL((fz_reduce_kernel<T, N1, N2, true>), dim3(P.red_wg), dim3(kBlock), lds, s, a);
  else
    hipLaunchKernelGGL((fz_reduce_kernel<T, N1, N2, false>), dim3(P.red_wg), dim3(kBlock), lds, s, a);
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
  if (P.unfused) return;
  const int M = P.M;
  if (!(M == 16 || M == 32 || M == 64 || M == 128 || M == 256)) return;
  if ((int)P.outs.size() > kOutPerThread * kBlock || P.outs.empty()) return;
  if ((int)P.terms.size() > kFMaxTerms || (int)P.qgroups.size() > kFMaxQ || P.nf2 > kFMaxComp ||
      (int)P.gcomp.size() > kFMaxComp)
    return;
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
