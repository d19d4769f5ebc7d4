// Device helpers over the operator geometry (Geo): fine-grid indices of the
// phases, collocation rows, and the spectra of A and Z* (section 3.2.2,
// Lemma 4.2; 2D section 5.2).  Shared by the power-of-two engine and the
// mixed-radix path.
#pragma once
#include "fft.h"
#include "internal.h"

namespace az {

__device__ __forceinline__ int64_t grid_index(const Geo& g, int ph, int64_t a, int64_t b) {
  if (g.dim == 1) return (int64_t)g.s * (a * g.N2 + b) + ph;
  const int rx = ph / g.s, ry = ph - rx * g.s;
  return ((int64_t)g.s * a + rx) * g.L + (int64_t)g.s * b + ry;
}

// The same with the oversampling factor as a compile-time constant (S == g.s)
// and the phase given by its coordinates (1D: rx = 0, ry = phase).
template <int S, bool D1>
__device__ __forceinline__ int64_t grid_index_s(const Geo& g, int rx, int ry, int64_t a, int64_t b) {
  if constexpr (D1) return (int64_t)S * (a * g.N2 + b) + ry;
  else return ((int64_t)S * a + rx) * g.L + (int64_t)S * b + ry;
}
template <bool D1>
__device__ __forceinline__ int64_t row_of_d(const Geo& g, int64_t gi) {
  if constexpr (D1) {
    const int64_t r = gi - g.i0;
    return (r >= 0 && r < g.M) ? r : -1;
  } else {
    return g.inv[gi];
  }
}

__device__ __forceinline__ int64_t row_of(const Geo& g, int64_t gi) {
  if (g.dim == 1) {
    const int64_t r = gi - g.i0;
    return (r >= 0 && r < g.M) ? r : -1;
  }
  return g.inv[gi];
}

// Unnormalised 2D spectrum of phase ph at frequency (ka, kb).
__device__ __forceinline__ double2 spec2d(const Geo& g, int ph, int ka, int kb) {
  const int rx = ph / g.s, ry = ph - rx * g.s;
  const int n1 = g.N1, n2 = g.N2;
  const double2 x0 = g.fac[rx * n1 + ka], y0 = g.facy[ry * n2 + kb];
  if (g.op == AZRBF_OP_APPROX) return cmul(x0, y0);
  const double2 x2 = g.fac[(g.s + rx) * n1 + ka], y2 = g.facy[(g.s + ry) * n2 + kb];
  const double2 d00 = cmul(x0, y0);
  double2 d = cadd(cadd(cmul(x2, y0), cmul(x0, y2)), cscale(d00, g.k2));
  return cscale(d, g.opscale);
}

// Engine kernels know the dimension at compile time (D1: 1D); the other
// dimension's code is then not compiled into them.
template <bool D1>
__device__ __forceinline__ double2 specA_d(const Geo& g, int ph, int ka, int kb) {
  if constexpr (D1) return g.spA[(int64_t)ph * g.N + (int64_t)ka * g.N2 + kb];
  else return cscale(spec2d(g, ph, ka, kb), 1.0 / (double)g.N);
}
template <bool D1>
__device__ __forceinline__ double2 specZ_d(const Geo& g, int ph, int ka, int kb) {
  if constexpr (D1) return g.spZ[(int64_t)ph * g.N + (int64_t)ka * g.N2 + kb];
  else return cscale(cconj(spec2d(g, ph, ka, kb)), g.w2[(int64_t)ka * g.N2 + kb]);
}

__device__ __forceinline__ double2 specA(const Geo& g, int ph, int ka, int kb) {
  if (g.dim == 1) return g.spA[(int64_t)ph * g.N + (int64_t)ka * g.N2 + kb];
  return cscale(spec2d(g, ph, ka, kb), 1.0 / (double)g.N);
}

__device__ __forceinline__ double2 specZ(const Geo& g, int ph, int ka, int kb) {
  if (g.dim == 1) return g.spZ[(int64_t)ph * g.N + (int64_t)ka * g.N2 + kb];
  return cscale(cconj(spec2d(g, ph, ka, kb)), g.w2[(int64_t)ka * g.N2 + kb]);
}

}  // namespace az
