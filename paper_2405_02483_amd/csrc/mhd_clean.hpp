// div B cleaning in Fourier space (Section 3, eq. clean1, eq. clean2):
// host-side view of mhd_clean.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "mhd_common.hpp"

namespace smhd {

// rocFFT plans per box shape and the scratch of the transforms; made on the
// first call (for the context's boxes and precision) and kept.
struct CleanState;
void clean_free(CleanState* s);

// Projects B (f.p[5..7]) of every box in place on the stream; the boxes
// must be periodic.  Returns 0, 1 (a rocFFT failure) or 2 (no memory),
// with a message in err.
template <class T>
int clean_boxes(CleanState** s, const std::vector<BoxDev>& boxes, P8<T> f, hipStream_t stream,
                std::string& err);

}  // namespace smhd
