// Specialised FFT passes of length 400 (see fft_fast_impl.h): the 2N of the
// 3D grids N = 200 used in the paper's 3D scattering runs (Table 7).
#include "fft_fast_impl.h"

namespace vg {
VG_FAST_INSTANTIATE(400, false)
}  // namespace vg
