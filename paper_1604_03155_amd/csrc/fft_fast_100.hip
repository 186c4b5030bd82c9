// Specialised FFT passes of length 100 (see fft_fast_impl.h): the 2N of the
// 3D grids N = 50 used in the paper's 3D scattering runs (Table 7).
#include "fft_fast_impl.h"

namespace vg {
VG_FAST_INSTANTIATE(100, false)
}  // namespace vg
