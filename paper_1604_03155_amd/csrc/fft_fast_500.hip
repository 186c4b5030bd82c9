// Specialised FFT passes of length 500 (see fft_fast_impl.h): the 2N of the
// 3D grids N = 250 used in the paper's 3D scattering runs (Table 7).
#include "fft_fast_impl.h"

namespace vg {
VG_FAST_INSTANTIATE(500, false)
}  // namespace vg
