// The 3j-weighted triple-product reduction (Sec. 4.2, eq. 41; Sec. 4.4, eq. 52):
//   B_mu(b1, b2) = N H / (I N_mode(b1) N_mode(b2) M^3)
//                  * sum_q sum_x Q_q(x; b1) f2_q(x; b2),
//   Q_q(x; b1)  = sum_t coef_t f1_t(x; b1) g_t(x),
// where the real fields f (parts of the F slots) and g (parts of the G grids)
// come from the inverse transforms and the terms (coef, f1, f2, g) are the
// real expansion of sum_{m1 m2 M} 3j F_l1^m1 F_l2^m2 G_L^M.
//
// Each workgroup walks a fixed set of cell chunks; a chunk's field values are
// staged in LDS, Q is formed in LDS, and every thread accumulates its outputs
// in FP64 registers. Per-workgroup partial sums are combined in a fixed order,
// so the result does not depend on scheduling.
#include "tsb_internal.h"

namespace tsb {

namespace {

constexpr int kOutPerThread = 16;   // outputs per thread per launch
constexpr int kRedMaxKinds = 32;    // F slot kinds and G grids of the matrix-core kernel

template <typename T>
struct RedArgs {
  typedef typename cplx<T>::type T2;
  const T2* fields;        // F slots [nb * nkinds][M^3] then G grids [ngrid][M^3]
  int64_t M3;
  int nb, nkinds, ngrid;
  int nfc, ngc, nq;
  const Component* fcomp;
  const Component* gcomp;
  const Term* terms;
  const QGroup* qg;
  const OutEntry* outs;
  int out0, nout;          // outputs [out0, out0 + nout) in this launch
  int nout_all;            // row length of partials
  int chunk;               // cells per chunk
  int64_t nchunks;
  double* partials;        // [nout_all][gridDim]
  // matrix-core kernel: per F slot kind and per G grid, the component taking
  // the real and the imaginary part (-1: none)
  int kre[kRedMaxKinds], kim[kRedMaxKinds], gre[kRedMaxKinds], gim[kRedMaxKinds];
};

template <typename T>
__global__ void __launch_bounds__(kBlock) reduce_kernel(RedArgs<T> a) {
  typedef typename cplx<T>::type T2;
  extern __shared__ char smem[];
  const int C = a.chunk;
  const int CP = C + 1;                          // odd row pitch: rows start in different banks
  T* Fv = (T*)smem;                              // [nb][nfc][CP]
  T* Gv = Fv + (size_t)a.nb * a.nfc * CP;        // [ngc][CP]
  T* Qv = Gv + (size_t)a.ngc * CP;               // [nq][nb][CP]
  const int tid = threadIdx.x;
  double acc[kOutPerThread];
#pragma unroll
  for (int r = 0; r < kOutPerThread; ++r) acc[r] = 0.0;

  for (int64_t ch = blockIdx.x; ch < a.nchunks; ch += gridDim.x) {
    const int64_t c0 = ch * C;
    // stage F slot parts: one complex load feeds up to two components
    const int nslot = a.nb * a.nkinds;
    for (int idx = tid; idx < nslot * C; idx += kBlock) {
      const int slot = idx / C, c = idx - slot * C;
      const T2 v = a.fields[(int64_t)slot * a.M3 + c0 + c];
      const int b = slot / a.nkinds, k = slot - b * a.nkinds;
      for (int f = 0; f < a.nfc; ++f)
        if (a.fcomp[f].slot == k) Fv[((size_t)b * a.nfc + f) * CP + c] = a.fcomp[f].part ? v.y : v.x;
    }
    for (int idx = tid; idx < a.ngrid * C; idx += kBlock) {
      const int g = idx / C, c = idx - g * C;
      const T2 v = a.fields[((int64_t)nslot + g) * a.M3 + c0 + c];
      for (int f = 0; f < a.ngc; ++f)
        if (a.gcomp[f].slot == g) Gv[(size_t)f * CP + c] = a.gcomp[f].part ? v.y : v.x;
    }
    __syncthreads();
    // Q_q(x; b1)
    for (int idx = tid; idx < a.nq * a.nb * C; idx += kBlock) {
      const int c = idx % C;
      const int qb = idx / C;
      const int b1 = qb % a.nb, q = qb / a.nb;
      const QGroup g = a.qg[q];
      double s = 0.0;
      for (int t = g.t0; t < g.t1; ++t) {
        const Term tm = a.terms[t];
        s += tm.coef * (double)Fv[((size_t)b1 * a.nfc + tm.f1) * CP + c] * (double)Gv[(size_t)tm.g * CP + c];
      }
      Qv[((size_t)q * a.nb + b1) * CP + c] = (T)s;
    }
    __syncthreads();
    // sum over the chunk's cells for every output of this thread
#pragma unroll
    for (int r = 0; r < kOutPerThread; ++r) {
      const int o = tid + r * kBlock;
      if (o >= a.nout) break;
      const OutEntry e = a.outs[a.out0 + o];
      double s = 0.0;
      for (int q = e.q0; q < e.q1; ++q) {
        const T* qr = Qv + ((size_t)q * a.nb + e.b1) * CP;
        const T* fr = Fv + ((size_t)e.b2 * a.nfc + a.qg[q].f2) * CP;
        for (int c = 0; c < C; ++c) s += (double)qr[c] * (double)fr[c];
      }
      acc[r] += s;
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < kOutPerThread; ++r) {
    const int o = tid + r * kBlock;
    if (o < a.nout) a.partials[(size_t)(a.out0 + o) * gridDim.x + blockIdx.x] = acc[r];
  }
}

// FP32 plans with at most 32 shells: the same staging and Q rows, but the sum
// over a chunk's cells of Q_q(x; b1) f2_q(x; b2) runs on the matrix cores as
// one 32 x 32 tile of (b1, b2) per Q group (FP32 32x32x2 MFMA; shells padded
// to 32, lanes past the shells feed zeros), FP32 within a chunk and FP64
// across chunks. Wavefront w holds the tiles of Q groups w, w + 4, ... (UPW
// of them); the workgroup's partial of every output is then formed from the
// tiles in a fixed order.
typedef float floatx16 __attribute__((ext_vector_type(16)));

template <int UPW>
__global__ void __launch_bounds__(kBlock) reduce_mfma_kernel(RedArgs<float> a) {
  extern __shared__ char smem[];
  const int C = a.chunk;
  const int CP = C + 1;
  float* Fv = (float*)smem;                      // [nb][nfc][CP]
  float* Gv = Fv + (size_t)a.nb * a.nfc * CP;    // [ngc][CP]
  float* Qv = Gv + (size_t)a.ngc * CP;           // [nq][nb][CP]
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  constexpr int kWaves = kBlock / 64;
  double acc[UPW][16];
#pragma unroll
  for (int u = 0; u < UPW; ++u)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[u][r] = 0.0;

  for (int64_t ch = blockIdx.x; ch < a.nchunks; ch += gridDim.x) {
    const int64_t c0 = ch * C;
    const int nslot = a.nb * a.nkinds;
    // one load per slot element, its parts straight to their component rows
    for (int idx = tid; idx < nslot * C; idx += kBlock) {
      const int slot = idx / C, c = idx - slot * C;
      const float2 v = a.fields[(int64_t)slot * a.M3 + c0 + c];
      const int b = slot / a.nkinds, k = slot - b * a.nkinds;
      const int fr = a.kre[k], fi = a.kim[k];
      if (fr >= 0) Fv[((size_t)b * a.nfc + fr) * CP + c] = v.x;
      if (fi >= 0) Fv[((size_t)b * a.nfc + fi) * CP + c] = v.y;
    }
    for (int idx = tid; idx < a.ngrid * C; idx += kBlock) {
      const int g = idx / C, c = idx - g * C;
      const float2 v = a.fields[((int64_t)nslot + g) * a.M3 + c0 + c];
      const int fr = a.gre[g], fi = a.gim[g];
      if (fr >= 0) Gv[(size_t)fr * CP + c] = v.x;
      if (fi >= 0) Gv[(size_t)fi * CP + c] = v.y;
    }
    __syncthreads();
    for (int idx = tid; idx < a.nq * a.nb * C; idx += kBlock) {
      const int c = idx % C;
      const int qb = idx / C;
      const int b1 = qb % a.nb, q = qb / a.nb;
      const QGroup g = a.qg[q];
      double s = 0.0;
      for (int t = g.t0; t < g.t1; ++t) {
        const Term tm = a.terms[t];
        s += tm.coef * (double)Fv[((size_t)b1 * a.nfc + tm.f1) * CP + c] * (double)Gv[(size_t)tm.g * CP + c];
      }
      Qv[((size_t)q * a.nb + b1) * CP + c] = (float)s;
    }
    __syncthreads();
    const int b = lane & 31, kh = lane >> 5;
    const bool live = b < a.nb;
#pragma unroll
    for (int u = 0; u < UPW; ++u) {
      const int q = wave + kWaves * u;
      if (q >= a.nq) break;   // uniform in the wavefront
      const float* qr = Qv + ((size_t)q * a.nb + (live ? b : 0)) * CP + kh;
      const float* fr = Fv + ((size_t)(live ? b : 0) * a.nfc + a.qg[q].f2) * CP + kh;
      floatx16 c = {};
      for (int kk = 0; kk < C; kk += 8) {
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
      for (int r = 0; r < 16; ++r) acc[u][r] += (double)c[r];
    }
    __syncthreads();   // the next chunk overwrites the staged rows
  }
  double* Ct = (double*)smem;   // [nq][32][32]
#pragma unroll
  for (int u = 0; u < UPW; ++u) {
    const int q = wave + kWaves * u;
    if (q >= a.nq) break;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3), j = lane & 31;
      Ct[((size_t)q * 32 + i) * 32 + j] = acc[u][r];
    }
  }
  __syncthreads();
  for (int o = tid; o < a.nout_all; o += kBlock) {
    const OutEntry e = a.outs[o];
    double v = 0.0;
    for (int q = e.q0; q < e.q1; ++q) v += Ct[((size_t)q * 32 + e.b1) * 32 + e.b2];
    a.partials[(size_t)o * gridDim.x + blockIdx.x] = v;
  }
}

// The same reduction for FP32 plans with at most 32 shells, 16 Q groups and 64
// terms, in workgroups of RB = 1024 threads (four wavefronts per SIMD with one
// workgroup per CU), or of 512 for at most 8 Q groups when two workgroups'
// staged rows fit the LDS of a CU (two interleaved chunk pipelines). The chunk
// length C is a template constant, so that every cell and slot index is a
// shift or a mask: each thread issues its share of a chunk's field loads
// before it stores any of them, as whole complex values into [slot][C] rows
// (F slots, then G grids, in their order in HBM); the Q rows are formed one
// group at a time from the (slot kind, part) and (grid, part) of each term in
// the kernel arguments (uniform loops, scalar loads), and one wavefront per Q
// group runs its 32 x 32 (b1, b2) tile on the matrix cores, reading the right
// factor's part from the staged rows. The arithmetic is that of
// reduce_mfma_kernel: Q in FP64 rounded to FP32, the products of a chunk
// summed in FP32, chunks in FP64.
constexpr int kRWLoads = 8;       // field loads per thread and chunk held in registers
constexpr int kRWTerms = 64, kRWQ = 16;

struct RedWideTables {
  double coef[kRWTerms];
  int f1k[kRWTerms], f1p[kRWTerms], gk[kRWTerms], gp[kRWTerms];   // slot kind / grid and part of each term
  int q_t0[kRWQ], q_t1[kRWQ], q_f2k[kRWQ], q_f2p[kRWQ];           // terms and right factor of each Q group
};

template <int kRWBlock, int kUnits, int kC>   // kUnits: Q groups per wavefront; kC: cells per chunk
__global__ void __launch_bounds__(kRWBlock, 4) reduce_mfma_wide_kernel(RedArgs<float> a, RedWideTables tb) {
  static_assert((kC & (kC - 1)) == 0 && kC >= 8 && kC <= 64, "chunk: a power of two in [8, 64]");
  constexpr int LC = kC == 8 ? 3 : (kC == 16 ? 4 : (kC == 32 ? 5 : 6));
  constexpr int CP = kC + 1;                     // row pitch (complex rows: odd in 8-byte units)
  extern __shared__ char smem[];
  const int nslot = a.nb * a.nkinds;
  const int nrow = nslot + a.ngrid;              // staged complex rows: F slots, then G grids
  float2* Sv = (float2*)smem;                    // [nrow][CP]
  float* Qv = (float*)(Sv + (size_t)nrow * CP);  // [nq][nb][CP]
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  double acc[kUnits][16];
#pragma unroll
  for (int u = 0; u < kUnits; ++u)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[u][r] = 0.0;
  const int nload = nrow << LC;                  // complex elements staged per chunk
  for (int64_t ch = blockIdx.x; ch < a.nchunks; ch += gridDim.x) {
    const float2* src = a.fields + (ch << LC);
    // every load of this thread first, then the stores
    for (int base = 0; base < nload; base += kRWLoads * kRWBlock) {
      float2 v[kRWLoads];
#pragma unroll
      for (int j = 0; j < kRWLoads; ++j) {
        const int idx = base + tid + j * kRWBlock;
        v[j] = make_float2(0.f, 0.f);
        if (idx < nload) v[j] = src[(int64_t)(idx >> LC) * a.M3 + (idx & (kC - 1))];
      }
#pragma unroll
      for (int j = 0; j < kRWLoads; ++j) {
        const int idx = base + tid + j * kRWBlock;
        if (idx < nload) Sv[(idx >> LC) * CP + (idx & (kC - 1))] = v[j];
      }
    }
    __syncthreads();
    // Q_q(x; b1), one group at a time: its terms are uniform across the workgroup
    for (int q = 0; q < a.nq; ++q) {
      const int t0 = tb.q_t0[q], t1 = tb.q_t1[q];
      for (int idx = tid; idx < (a.nb << LC); idx += kRWBlock) {
        const int b1 = idx >> LC, c = idx & (kC - 1);
        const float* frow = (const float*)(Sv + (size_t)b1 * a.nkinds * CP + c);
        const float* grow = (const float*)(Sv + (size_t)nslot * CP + c);
        double s = 0.0;
        for (int t = t0; t < t1; ++t)
          s += tb.coef[t] * (double)frow[2 * tb.f1k[t] * CP + tb.f1p[t]] * (double)grow[2 * tb.gk[t] * CP + tb.gp[t]];
        Qv[((size_t)q * a.nb + b1) * CP + c] = (float)s;
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kUnits; ++u) {
      const int q = wave + u * (kRWBlock / 64);
      if (q >= a.nq) break;   // uniform in the wavefront
      const int b = lane & 31, kh = lane >> 5;
      const bool live = b < a.nb;
      const float* qr = Qv + ((size_t)q * a.nb + (live ? b : 0)) * CP + kh;
      const float* fr = (const float*)(Sv + ((size_t)(live ? b : 0) * a.nkinds + tb.q_f2k[q]) * CP + kh) + tb.q_f2p[q];
      floatx16 c = {};
      for (int kk = 0; kk < kC; kk += 8) {
        float av[4], bv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          av[j] = live ? qr[kk + 2 * j] : 0.f;
          bv[j] = live ? fr[2 * (kk + 2 * j)] : 0.f;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) c = __builtin_amdgcn_mfma_f32_32x32x2f32(av[j], bv[j], c, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[u][r] += (double)c[r];
    }
    __syncthreads();   // the next chunk overwrites the staged rows
  }
  double* Ct = (double*)smem;   // [nq][32][32]
#pragma unroll
  for (int u = 0; u < kUnits; ++u) {
    const int q = wave + u * (kRWBlock / 64);
    if (q >= a.nq) break;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3), j = lane & 31;
      Ct[((size_t)q * 32 + i) * 32 + j] = acc[u][r];
    }
  }
  __syncthreads();
  for (int o = tid; o < a.nout_all; o += kRWBlock) {
    const OutEntry e = a.outs[o];
    double v = 0.0;
    for (int q = e.q0; q < e.q1; ++q) v += Ct[((size_t)q * 32 + e.b1) * 32 + e.b2];
    a.partials[(size_t)o * gridDim.x + blockIdx.x] = v;
  }
}

// One block per output: each thread sums a fixed subset of the workgroup
// partials, then a fixed-shape tree; the order never depends on scheduling.
__global__ void __launch_bounds__(kBlock) reduce_final_kernel(const double* partials, int nwg,
                                                              const double* norm, const DevScalars* scal,
                                                              double* B) {
  __shared__ double sh[kBlock];
  const int o = blockIdx.x;
  const double* row = partials + (size_t)o * nwg;
  double s = 0.0;
  for (int w = threadIdx.x; w < nwg; w += kBlock) s += row[w];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int st = kBlock / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) B[o] = sh[0] * norm[o] / scal->I;
}

template <typename T>
int reduce_impl(Plan& P, hipStream_t s) {
  typedef typename cplx<T>::type T2;
  RedArgs<T> a{};
  a.fields = (const T2*)P.d_fields;   // F slots at 0, G grids at P.g_offset
  a.M3 = (int64_t)P.M * P.M * P.M;
  a.nb = P.nb;
  a.nkinds = (int)P.fkinds.size();
  a.ngrid = (int)P.grids.size();
  a.nfc = (int)P.fcomp.size();
  a.ngc = (int)P.gcomp.size();
  a.nq = (int)P.qgroups.size();
  a.fcomp = P.d_fcomp;
  a.gcomp = P.d_gcomp;
  a.terms = P.d_terms;
  a.qg = P.d_qgroups;
  a.outs = P.d_outs;
  a.chunk = P.red_chunk;
  a.nchunks = a.M3 / P.red_chunk;
  a.partials = P.d_partials;
  const size_t lds = sizeof(T) * (size_t)(P.red_chunk + 1) *
                     ((size_t)a.nb * a.nfc + a.ngc + (size_t)a.nq * a.nb);
  const int nout_all = (int)P.outs.size();
  const int per_launch = kOutPerThread * kBlock;
  a.nout_all = nout_all;
  prof_begin(P, kStReduce, s);
  if constexpr (std::is_same<T, float>::value) {
    if (P.red_mfma > 0) {
      const size_t lds_m = std::max(lds, (size_t)a.nq * 32 * 32 * sizeof(double));
      for (int k = 0; k < kRedMaxKinds; ++k) a.kre[k] = a.kim[k] = a.gre[k] = a.gim[k] = -1;
      for (size_t f = 0; f < P.fcomp.size(); ++f) (P.fcomp[f].part ? a.kim : a.kre)[P.fcomp[f].slot] = (int)f;
      for (size_t f = 0; f < P.gcomp.size(); ++f) (P.gcomp[f].part ? a.gim : a.gre)[P.gcomp[f].slot] = (int)f;
      a.out0 = 0;
      a.nout = nout_all;
      if (P.red_mfma == 8) {
        RedWideTables tb{};
        for (size_t t = 0; t < P.terms.size(); ++t) {
          tb.coef[t] = P.terms[t].coef;
          tb.f1k[t] = P.fcomp[P.terms[t].f1].slot;
          tb.f1p[t] = P.fcomp[P.terms[t].f1].part;
          tb.gk[t] = P.gcomp[P.terms[t].g].slot;
          tb.gp[t] = P.gcomp[P.terms[t].g].part;
        }
        for (size_t q = 0; q < P.qgroups.size(); ++q) {
          tb.q_t0[q] = P.qgroups[q].t0;
          tb.q_t1[q] = P.qgroups[q].t1;
          tb.q_f2k[q] = P.fcomp[P.qgroups[q].f2].slot;
          tb.q_f2p[q] = P.fcomp[P.qgroups[q].f2].part;
        }
        const size_t lds_w = std::max<size_t>((size_t)reduce_lds_bytes(P), (size_t)a.nq * 32 * 32 * sizeof(double));
        const bool pair = P.red_block == 512 && a.nq <= 8;
        const dim3 grid(P.red_wg), block(pair ? 512 : 1024);
        switch (P.red_chunk) {
#define TSB_RW(C)                                                                              \
  case C:                                                                                      \
    if (pair)                                                                                  \
      hipLaunchKernelGGL((reduce_mfma_wide_kernel<512, 1, C>), grid, block, lds_w, s, a, tb);  \
    else                                                                                       \
      hipLaunchKernelGGL((reduce_mfma_wide_kernel<1024, 1, C>), grid, block, lds_w, s, a, tb); \
    break;
          TSB_RW(8)
          TSB_RW(16)
          TSB_RW(32)
          TSB_RW(64)
#undef TSB_RW
          default:
            return fail(TSB_E_UNSUPPORTED, "matrix-core reduction: chunk length not 8, 16, 32 or 64");
        }
        prof_end(P, kStReduce, s);
        TSB_HIP(hipGetLastError());
        return run_reduce_final(P, s);
      }
      if (P.red_mfma == 1)
        hipLaunchKernelGGL(reduce_mfma_kernel<1>, dim3(P.red_wg), dim3(kBlock), lds_m, s, a);
      else if (P.red_mfma == 2)
        hipLaunchKernelGGL(reduce_mfma_kernel<2>, dim3(P.red_wg), dim3(kBlock), lds_m, s, a);
      else
        hipLaunchKernelGGL(reduce_mfma_kernel<4>, dim3(P.red_wg), dim3(kBlock), lds_m, s, a);
      prof_end(P, kStReduce, s);
      TSB_HIP(hipGetLastError());
      return run_reduce_final(P, s);
    }
  }
  for (int o0 = 0; o0 < nout_all; o0 += per_launch) {
    a.out0 = o0;
    a.nout = std::min(per_launch, nout_all - o0);
    hipLaunchKernelGGL(reduce_kernel<T>, dim3(P.red_wg), dim3(kBlock), lds, s, a);
  }
  prof_end(P, kStReduce, s);
  TSB_HIP(hipGetLastError());
  return run_reduce_final(P, s);
}

}  // namespace

int64_t reduce_lds_bytes(const Plan& P) {
  const int64_t esz = P.precision == TSB_FP64 ? 8 : 4;
  if (P.red_mfma == 8)   // complex rows of every F slot and G grid, then the Q rows
    return 4 * (P.red_chunk + 1) * (2 * ((int64_t)P.nb * (int64_t)P.fkinds.size() + (int64_t)P.grids.size()) +
                                    (int64_t)P.qgroups.size() * P.nb);
  return esz * (P.red_chunk + 1) *
         ((int64_t)P.nb * (int64_t)P.fcomp.size() + (int64_t)P.gcomp.size() + (int64_t)P.qgroups.size() * P.nb);
}

bool reduce_pair_fits(const Plan& P) {
  const int64_t lds = std::max<int64_t>(reduce_lds_bytes(P), (int64_t)P.qgroups.size() * 32 * 32 * 8);
  return P.red_mfma == 8 && P.qgroups.size() <= 8 && 2 * lds <= 160 * 1024;
}

int run_reduce_final(Plan& P, hipStream_t s) {
  const int nout_all = (int)P.outs.size();
  if (nout_all == 0) return TSB_OK;
  prof_begin(P, kStReduceFinal, s);
  hipLaunchKernelGGL(reduce_final_kernel, dim3(nout_all), dim3(kBlock), 0, s, (const double*)P.d_partials,
                     P.red_wg, (const double*)P.d_out_norm, (const DevScalars*)P.d_scal, P.d_B);
  prof_end(P, kStReduceFinal, s);
  TSB_HIP(hipGetLastError());
  return TSB_OK;
}

namespace {

__global__ void __launch_bounds__(kBlock) fill_nan_kernel(double* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
    p[i] = __longlong_as_double(0x7ff8000000000000LL);   // quiet NaN
}

__global__ void __launch_bounds__(kBlock) scatter_outputs_kernel(const double* B, const OutEntry* outs, int nout,
                                                                int nb, double* full) {
  for (int o = blockIdx.x * kBlock + threadIdx.x; o < nout; o += gridDim.x * kBlock) {
    const OutEntry e = outs[o];
    full[((int64_t)e.mu * nb + e.b1) * nb + e.b2] = B[o];
  }
}

}  // namespace

// The computed outputs in the caller's [n_mult][n_bins][n_bins] layout, NaN
// where no pair is computed, written to device memory `full`.
int run_scatter_outputs(Plan& P, double* full, hipStream_t s) {
  const int64_t total = (int64_t)P.mult.size() * P.nb * P.nb;
  hipLaunchKernelGGL(fill_nan_kernel, dim3((int)std::min<int64_t>((total + kBlock - 1) / kBlock, 1024)),
                     dim3(kBlock), 0, s, full, total);
  const int nout = (int)P.outs.size();
  if (nout > 0)
    hipLaunchKernelGGL(scatter_outputs_kernel, dim3((nout + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
                       (const double*)P.d_B, (const OutEntry*)P.d_outs, nout, P.nb, full);
  TSB_HIP(hipGetLastError());
  return TSB_OK;
}

int run_reduce(Plan& P, hipStream_t s) {
  if (P.outs.empty()) return TSB_OK;
  return P.precision == TSB_FP64 ? reduce_impl<double>(P, s) : reduce_impl<float>(P, s);
}

}  // namespace tsb
