// heat1d_weights.h -- host-side weights of the fused S-step sweeps (no device
// code: the C ABI reports them, the kernels receive them as arguments).
#pragma once

#include <cmath>

namespace heat1d {

// Weights w[0..S] of the S-step stencil u_i <- w_0 u_i + sum_{d=1..S} w_d
// (u_{i-d} + u_{i+d}), which stands for S steps of Eq.3 (Section 2) on points
// at least S away from a rod end.
template <typename F>
struct StepWeights {
  F w[9];  // w[0..S]
};

// Weights of the S-step stencil: coefficients of (r, 1-2r, r)^S, formed from
// the same r the single steps use (r rounded to F), so that the interior and
// the end tiles of one run iterate the same operator.
//
// The S-step operator of Eq.3 has row sum exactly 1 (it maps a constant state
// to itself).  Rounding each weight to F on its own breaks that: the rounded
// row sum 1 + delta scales the slowly decaying content by (1 + delta) per
// sweep, a drift that grows as K/S * delta and is far larger than the
// unbiased rounding of the sweeps themselves (about 3e-5 after 2000 FP32
// steps at r = 0.41, S = 2).  Instead the off-centre weights are rounded to
// the grid of multiples of 2^-(p+1) (p = 24 bits for FP32, 53 for FP64) and
// the centre weight is w0 = 1 - 2 (w1 + ... + wS), which then is a multiple
// of 2^-p in (0, 1] and so exact in F: the row sum is exactly 1.  The grid
// moves a weight by at most 2^-(p+2); such a change that keeps the row sum
// alters the per-sweep factor of a Fourier mode of angle t by at most
// sum_d 2 |dw_d| (1 - cos dt), second order in t for the slow modes that
// survive many sweeps.
inline void step_weights_exact(double r, int S, int mantissa_bits, double* w) {
  double c[17] = {1.0};  // polynomial in x, centre at index S
  int len = 1;
  for (int k = 0; k < S; ++k) {
    double n[17] = {0.0};
    for (int i = 0; i < len; ++i) {
      n[i] += r * c[i];
      n[i + 1] += (1.0 - 2.0 * r) * c[i];
      n[i + 2] += r * c[i];
    }
    len += 2;
    for (int i = 0; i < len; ++i) c[i] = n[i];
  }
  const double grid = std::ldexp(1.0, -(mantissa_bits + 1));
  double off = 0.0;  // w1 + ... + wS, exact: multiples of the grid below 1/2
  for (int d = 1; d <= S; ++d) {
    w[d] = std::nearbyint(c[S + d] / grid) * grid;
    off += w[d];
  }
  w[0] = 1.0 - 2.0 * off;  // exact: a multiple of 2^-p in (0, 1]
}

template <typename F>
inline StepWeights<F> step_weights(double r, int S) {
  constexpr int bits = sizeof(F) == 4 ? 24 : 53;
  double w[9] = {1.0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (S > 1) step_weights_exact((double)(F)r, S, bits, w);
  StepWeights<F> sw{};
  for (int d = 0; d <= S && d < 9; ++d) sw.w[d] = (F)w[d];
  return sw;
}

}  // namespace heat1d
