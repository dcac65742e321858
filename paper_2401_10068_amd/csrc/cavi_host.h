// Host-side helpers shared by the C ABI sources (cavi_api.cpp, cavi_static.hip).  Not part of
// the public ABI.
#pragma once

#include <stdint.h>

#include <vector>

#include "../../include/cavi.h"
#include "cavi_impl.h"

namespace cavi {

constexpr int kHistSingle = 4096;  // bounds kept by a single-dataset handle

// Record the text of an error for cavi_last_error() and return st.
cavi_status fail(cavi_status st, const char *fmt, ...);

bool finite_pos(double v);

// Shape of a batch of B datasets (rows N[b], subpopulations K[b], G genes); ds (optional)
// receives the per-dataset table.  CAVI_E_INVAL for sizes out of range.
cavi_status make_shape(int32_t B, const int64_t *N, const int32_t *K, int32_t G, int hist_cap, Shape &s,
                       std::vector<Ds> *ds);

// The prior (NULL: the defaults) checked and converted.
cavi_status check_prior(const cavi_prior *prior, Prior &p);

}  // namespace cavi

#define HIPCHK(expr)                                                                                \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess) return cavi::fail(CAVI_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)
