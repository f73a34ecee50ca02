// In-register power-of-two DFTs shared by the FFT passes and the fused
// z-pass + reduction.
#pragma once

#include "tsb_internal.h"

namespace tsb {
namespace {

// e^{-2 pi i j/32}, j < 32: twiddles of the in-register transforms (R <= 32).
// constexpr: with the unrolled loops every index is a constant, so each
// twiddle becomes an immediate operand of the working precision.
constexpr double kW32[32][2] = {
    {1.0, -0.0}, {0.98078528040323043, -0.19509032201612825}, {0.92387953251128674, -0.38268343236508978},
    {0.83146961230254524, -0.55557023301960218}, {0.70710678118654757, -0.70710678118654746},
    {0.55557023301960229, -0.83146961230254524}, {0.38268343236508984, -0.92387953251128674},
    {0.19509032201612833, -0.98078528040323043}, {0.0, -1.0}, {-0.19509032201612819, -0.98078528040323043},
    {-0.38268343236508973, -0.92387953251128674}, {-0.55557023301960196, -0.83146961230254546},
    {-0.70710678118654746, -0.70710678118654757}, {-0.83146961230254535, -0.55557023301960218},
    {-0.92387953251128674, -0.38268343236508989}, {-0.98078528040323043, -0.19509032201612861},
    {-1.0, -0.0}, {-0.98078528040323043, 0.19509032201612836}, {-0.92387953251128685, 0.38268343236508967},
    {-0.83146961230254546, 0.55557023301960196}, {-0.70710678118654768, 0.70710678118654746},
    {-0.55557023301960218, 0.83146961230254524}, {-0.38268343236509034, 0.92387953251128652},
    {-0.19509032201612866, 0.98078528040323032}, {0.0, 1.0}, {0.19509032201612828, 0.98078528040323043},
    {0.38268343236509, 0.92387953251128663}, {0.55557023301960184, 0.83146961230254546},
    {0.70710678118654735, 0.70710678118654768}, {0.83146961230254524, 0.55557023301960218},
    {0.92387953251128652, 0.38268343236509039}, {0.98078528040323032, 0.19509032201612872}};

// In-register radix-2 decimation-in-frequency DFT of R points (R a power of 2,
// R <= 32); dir -1 forward, +1 inverse. On return v[i] holds output index
// bitrev_R(i).
template <typename T, typename T2, int R>
__device__ inline void reg_fft(T2 (&v)[R], int dir) {
#pragma unroll
  for (int s = R / 2; s >= 1; s /= 2) {
#pragma unroll
    for (int blk = 0; blk < R; blk += 2 * s) {
#pragma unroll
      for (int j = 0; j < s; ++j) {
        const T2 x = v[blk + j], y = v[blk + j + s];
        T2 sum, d;
        sum.x = x.x + y.x;
        sum.y = x.y + y.y;
        d.x = x.x - y.x;
        d.y = x.y - y.y;
        v[blk + j] = sum;
        if (j == 0) {
          v[blk + j + s] = d;
        } else {
          const int t = j * (32 / (2 * s));       // W_{2s}^j = W_32^{j 32/(2s)}
          const T wr = (T)kW32[t][0];
          const T wi = (T)(dir < 0 ? kW32[t][1] : -kW32[t][1]);
          T2 o;
          o.x = d.x * wr - d.y * wi;
          o.y = d.x * wi + d.y * wr;
          v[blk + j + s] = o;
        }
      }
    }
  }
}

template <int R>
__host__ __device__ constexpr int bit_reverse(int i) {
  int r = 0;
  for (int b = 1; b < R; b <<= 1) {
    r = (r << 1) | (i & 1);
    i >>= 1;
  }
  return r;
}

}  // namespace
}  // namespace tsb
