// Specialised FFT passes of length 1024 (see fft_fast_impl.h).
#include "fft_fast_impl.h"

namespace vg {
VG_FAST_INSTANTIATE(1024, false)
}  // namespace vg
