// FP64 special functions for the conjugate updates and the lower bound on
// the device, for arguments x > 0.
//
// lgamma: shift x up to >= 8 with ln G(x) = ln G(x + n) - ln(x (x+1) ... (x+n-1))
// (one log of the product), then Stirling's series
//   ln G(x) = (x - 1/2) ln x - x + ln(2 pi)/2 + sum_k B_2k / (2k (2k-1) x^(2k-1))
// (Abramowitz & Stegun 6.1.40-6.1.41), terms through x^-13.
// digamma: shift x up to >= 12 with psi(x) = psi(x + 1) - 1/x, then
//   psi(x) = ln x - 1/(2x) - sum_k B_2k / (2k x^2k)   (A&S 6.3.18), terms through x^-12.
#pragma once

#include <hip/hip_runtime.h>

namespace cavi {

__device__ __forceinline__ double dev_lgamma(double x)
{
    double prod = 1.0;
    while (x < 8.0) {
        prod *= x;
        x += 1.0;
    }
    const double r = 1.0 / x;
    const double r2 = r * r;
    // B2/2 = 1/12, B4/12 = -1/360, B6/30 = 1/1260, B8/56 = -1/1680,
    // B10/90 = 1/1188, B12/132 = -691/360360, B14/182 = 1/156
    double s = 1.0 / 156.0;
    s = s * r2 - 691.0 / 360360.0;
    s = s * r2 + 1.0 / 1188.0;
    s = s * r2 - 1.0 / 1680.0;
    s = s * r2 + 1.0 / 1260.0;
    s = s * r2 - 1.0 / 360.0;
    s = s * r2 + 1.0 / 12.0;
    const double half_ln_2pi = 0.91893853320467274178032973640562;
    return (x - 0.5) * log(x) - x + half_ln_2pi + s * r - log(prod);
}

__device__ __forceinline__ double dev_digamma(double x)
{
    double shift = 0.0;
    while (x < 12.0) {
        shift += 1.0 / x;
        x += 1.0;
    }
    const double r2 = 1.0 / (x * x);
    // B2/2 = 1/12, B4/4 = -1/120, B6/6 = 1/252, B8/8 = -1/240,
    // B10/10 = 1/132, B12/12 = -691/32760
    double s = -691.0 / 32760.0;
    s = s * r2 + 1.0 / 132.0;
    s = s * r2 - 1.0 / 240.0;
    s = s * r2 + 1.0 / 252.0;
    s = s * r2 - 1.0 / 120.0;
    s = s * r2 + 1.0 / 12.0;
    return log(x) - 0.5 / x - s * r2 - shift;
}

}  // namespace cavi
