// Specialised FFT passes of length 64 (see fft_fast_impl.h).
#include "fft_fast_impl.h"

namespace vg {
VG_FAST_INSTANTIATE(64, false)
}  // namespace vg
