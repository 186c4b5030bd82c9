// Dispatch of the length-specialised FFT passes (kernels in fft_fast_impl.h,
// one translation unit per length).
#include "common.h"

namespace vg {

int fast_C_32(int mode, bool fp64);
hipError_t launch_fast_32(const PassDesc& p, int mode, int kind, bool fp64, hipStream_t s);
int fast_C_64(int mode, bool fp64);
hipError_t launch_fast_64(const PassDesc& p, int mode, int kind, bool fp64, hipStream_t s);
int fast_C_96(int mode, bool fp64);
hipError_t launch_fast_96(const PassDesc& p, int mode, int kind, bool fp64, hipStream_t s);
int fast_C_128(int mode, bool fp64);
hipError_t launch_fast_128(const PassDesc& p, int mode, int kind, bool fp64, hipStream_t s);
int fast_C_192(int mode, bool fp64);
hipError_t launch_fast_192(const PassDesc& p, int mode, int kind, bool fp64, hipStream_t s);
int fast_C_256(int mode, bool fp64);
hipError_t launch_fast_256(const PassDesc& p, int mode, int kind, bool fp64, hipStream_t s);
int fast_C_512(int mode, bool fp64);
hipError_t launch_fast_512(const PassDesc& p, int mode, int kind, bool fp64, hipStream_t s);
int fast_C_1024(int mode, bool fp64);
hipError_t launch_fast_1024(const PassDesc& p, int mode, int kind, bool fp64, hipStream_t s);
int fast_C_2048(int mode, bool fp64);
hipError_t launch_fast_2048(const PassDesc& p, int mode, int kind, bool fp64, hipStream_t s);
int fast_C_4096(int mode, bool fp64);
hipError_t launch_fast_4096(const PassDesc& p, int mode, int kind, bool fp64, hipStream_t s);
int fast_C_8192(int mode, bool fp64);
hipError_t launch_fast_8192(const PassDesc& p, int mode, int kind, bool fp64, hipStream_t s);
int fast_C_100(int mode, bool fp64);
hipError_t launch_fast_100(const PassDesc& p, int mode, int kind, bool fp64, hipStream_t s);
int fast_C_200(int mode, bool fp64);
hipError_t launch_fast_200(const PassDesc& p, int mode, int kind, bool fp64, hipStream_t s);
int fast_C_400(int mode, bool fp64);
hipError_t launch_fast_400(const PassDesc& p, int mode, int kind, bool fp64, hipStream_t s);
int fast_C_500(int mode, bool fp64);
hipError_t launch_fast_500(const PassDesc& p, int mode, int kind, bool fp64, hipStream_t s);
int fast_C_300(int mode, bool fp64);
hipError_t launch_fast_300(const PassDesc& p, int mode, int kind, bool fp64, hipStream_t s);
int fast_C_3200(int mode, bool fp64);
hipError_t launch_fast_3200(const PassDesc& p, int mode, int kind, bool fp64, hipStream_t s);
int fast_C_6400(int mode, bool fp64);
hipError_t launch_fast_6400(const PassDesc& p, int mode, int kind, bool fp64, hipStream_t s);
int fast_C_12800(int mode, bool fp64);
hipError_t launch_fast_12800(const PassDesc& p, int mode, int kind, bool fp64, hipStream_t s);

// (declarations of the per-length offset checks)
bool fast_fits_32(int mode, bool fp64, long long ise, long long ose, long long iiq, long long oiq);
bool fast_fits_64(int mode, bool fp64, long long ise, long long ose, long long iiq, long long oiq);
bool fast_fits_96(int mode, bool fp64, long long ise, long long ose, long long iiq, long long oiq);
bool fast_fits_128(int mode, bool fp64, long long ise, long long ose, long long iiq, long long oiq);
bool fast_fits_192(int mode, bool fp64, long long ise, long long ose, long long iiq, long long oiq);
bool fast_fits_256(int mode, bool fp64, long long ise, long long ose, long long iiq, long long oiq);
bool fast_fits_512(int mode, bool fp64, long long ise, long long ose, long long iiq, long long oiq);
bool fast_fits_1024(int mode, bool fp64, long long ise, long long ose, long long iiq, long long oiq);
bool fast_fits_2048(int mode, bool fp64, long long ise, long long ose, long long iiq, long long oiq);
bool fast_fits_4096(int mode, bool fp64, long long ise, long long ose, long long iiq, long long oiq);
bool fast_fits_8192(int mode, bool fp64, long long ise, long long ose, long long iiq, long long oiq);
bool fast_fits_100(int mode, bool fp64, long long ise, long long ose, long long iiq, long long oiq);
bool fast_fits_200(int mode, bool fp64, long long ise, long long ose, long long iiq, long long oiq);
bool fast_fits_400(int mode, bool fp64, long long ise, long long ose, long long iiq, long long oiq);
bool fast_fits_500(int mode, bool fp64, long long ise, long long ose, long long iiq, long long oiq);
bool fast_fits_300(int mode, bool fp64, long long ise, long long ose, long long iiq, long long oiq);
bool fast_fits_3200(int mode, bool fp64, long long ise, long long ose, long long iiq, long long oiq);
bool fast_fits_6400(int mode, bool fp64, long long ise, long long ose, long long iiq, long long oiq);
bool fast_fits_12800(int mode, bool fp64, long long ise, long long ose, long long iiq, long long oiq);

// Pencils per workgroup the specialised kernel uses for (L, mode, precision),
// or 0 when no specialisation exists (the generic kernel is used).
int fast_pass_C(int L, int mode, bool fp64) {
    switch (L) {
        case 32: return fast_C_32(mode, fp64);
        case 64: return fast_C_64(mode, fp64);
        case 96: return fast_C_96(mode, fp64);
        case 128: return fast_C_128(mode, fp64);
        case 192: return fast_C_192(mode, fp64);
        case 256: return fast_C_256(mode, fp64);
        case 512: return fast_C_512(mode, fp64);
        case 1024: return fast_C_1024(mode, fp64);
        case 2048: return fast_C_2048(mode, fp64);
        case 4096: return fast_C_4096(mode, fp64);
        case 8192: return fast_C_8192(mode, fp64);
        case 100: return fast_C_100(mode, fp64);
        case 200: return fast_C_200(mode, fp64);
        case 400: return fast_C_400(mode, fp64);
        case 500: return fast_C_500(mode, fp64);
        case 300: return fast_C_300(mode, fp64);
        case 3200: return fast_C_3200(mode, fp64);
        case 6400: return fast_C_6400(mode, fp64);
        case 12800: return fast_C_12800(mode, fp64);
        default: return 0;
    }
}

// Whether the specialised kernel's 32-bit lane offsets cover these strides.
bool fast_pass_fits(int L, int mode, bool fp64, long long ise, long long ose, long long iiq, long long oiq) {
    switch (L) {
        case 32: return fast_fits_32(mode, fp64, ise, ose, iiq, oiq);
        case 64: return fast_fits_64(mode, fp64, ise, ose, iiq, oiq);
        case 96: return fast_fits_96(mode, fp64, ise, ose, iiq, oiq);
        case 128: return fast_fits_128(mode, fp64, ise, ose, iiq, oiq);
        case 192: return fast_fits_192(mode, fp64, ise, ose, iiq, oiq);
        case 256: return fast_fits_256(mode, fp64, ise, ose, iiq, oiq);
        case 512: return fast_fits_512(mode, fp64, ise, ose, iiq, oiq);
        case 1024: return fast_fits_1024(mode, fp64, ise, ose, iiq, oiq);
        case 2048: return fast_fits_2048(mode, fp64, ise, ose, iiq, oiq);
        case 4096: return fast_fits_4096(mode, fp64, ise, ose, iiq, oiq);
        case 8192: return fast_fits_8192(mode, fp64, ise, ose, iiq, oiq);
        case 100: return fast_fits_100(mode, fp64, ise, ose, iiq, oiq);
        case 200: return fast_fits_200(mode, fp64, ise, ose, iiq, oiq);
        case 400: return fast_fits_400(mode, fp64, ise, ose, iiq, oiq);
        case 500: return fast_fits_500(mode, fp64, ise, ose, iiq, oiq);
        case 300: return fast_fits_300(mode, fp64, ise, ose, iiq, oiq);
        case 3200: return fast_fits_3200(mode, fp64, ise, ose, iiq, oiq);
        case 6400: return fast_fits_6400(mode, fp64, ise, ose, iiq, oiq);
        case 12800: return fast_fits_12800(mode, fp64, ise, ose, iiq, oiq);
        default: return false;
    }
}

hipError_t launch_fast_pass(const PassDesc& p, int mode, int kind, bool fp64, hipStream_t s) {
    switch (p.L) {
        case 32: return launch_fast_32(p, mode, kind, fp64, s);
        case 64: return launch_fast_64(p, mode, kind, fp64, s);
        case 96: return launch_fast_96(p, mode, kind, fp64, s);
        case 128: return launch_fast_128(p, mode, kind, fp64, s);
        case 192: return launch_fast_192(p, mode, kind, fp64, s);
        case 256: return launch_fast_256(p, mode, kind, fp64, s);
        case 512: return launch_fast_512(p, mode, kind, fp64, s);
        case 1024: return launch_fast_1024(p, mode, kind, fp64, s);
        case 2048: return launch_fast_2048(p, mode, kind, fp64, s);
        case 4096: return launch_fast_4096(p, mode, kind, fp64, s);
        case 8192: return launch_fast_8192(p, mode, kind, fp64, s);
        case 100: return launch_fast_100(p, mode, kind, fp64, s);
        case 200: return launch_fast_200(p, mode, kind, fp64, s);
        case 400: return launch_fast_400(p, mode, kind, fp64, s);
        case 500: return launch_fast_500(p, mode, kind, fp64, s);
        case 300: return launch_fast_300(p, mode, kind, fp64, s);
        case 3200: return launch_fast_3200(p, mode, kind, fp64, s);
        case 6400: return launch_fast_6400(p, mode, kind, fp64, s);
        case 12800: return launch_fast_12800(p, mode, kind, fp64, s);
        default: return hipErrorInvalidValue;
    }
}

// grouped kernels
hipError_t launch_fast_group_32(const PassDesc& proto, const GroupArgs& g, int mode, int kind, bool fp64, hipStream_t s);
hipError_t launch_fast_group_64(const PassDesc& proto, const GroupArgs& g, int mode, int kind, bool fp64, hipStream_t s);
hipError_t launch_fast_group_96(const PassDesc& proto, const GroupArgs& g, int mode, int kind, bool fp64, hipStream_t s);
hipError_t launch_fast_group_128(const PassDesc& proto, const GroupArgs& g, int mode, int kind, bool fp64, hipStream_t s);
hipError_t launch_fast_group_192(const PassDesc& proto, const GroupArgs& g, int mode, int kind, bool fp64, hipStream_t s);
hipError_t launch_fast_group_256(const PassDesc& proto, const GroupArgs& g, int mode, int kind, bool fp64, hipStream_t s);
hipError_t launch_fast_group_512(const PassDesc& proto, const GroupArgs& g, int mode, int kind, bool fp64, hipStream_t s);
hipError_t launch_fast_group_1024(const PassDesc& proto, const GroupArgs& g, int mode, int kind, bool fp64, hipStream_t s);
hipError_t launch_fast_group_100(const PassDesc& proto, const GroupArgs& g, int mode, int kind, bool fp64, hipStream_t s);
hipError_t launch_fast_group_200(const PassDesc& proto, const GroupArgs& g, int mode, int kind, bool fp64, hipStream_t s);
hipError_t launch_fast_group_400(const PassDesc& proto, const GroupArgs& g, int mode, int kind, bool fp64, hipStream_t s);
hipError_t launch_fast_group_500(const PassDesc& proto, const GroupArgs& g, int mode, int kind, bool fp64, hipStream_t s);

bool fast_group_supported(int L) {
    return L == 32 || L == 64 || L == 96 || L == 100 || L == 128 || L == 192 || L == 200 || L == 256 || L == 400 ||
           L == 500 || L == 512 || L == 1024;
}

hipError_t launch_fast_group(const PassDesc& proto, const GroupArgs& g, int mode, int kind, bool fp64, hipStream_t s) {
    if (g.nitems <= 0 || g.ntiles == 0) return hipSuccess;
    switch (proto.L) {
        case 32: return launch_fast_group_32(proto, g, mode, kind, fp64, s);
        case 64: return launch_fast_group_64(proto, g, mode, kind, fp64, s);
        case 96: return launch_fast_group_96(proto, g, mode, kind, fp64, s);
        case 128: return launch_fast_group_128(proto, g, mode, kind, fp64, s);
        case 192: return launch_fast_group_192(proto, g, mode, kind, fp64, s);
        case 256: return launch_fast_group_256(proto, g, mode, kind, fp64, s);
        case 512: return launch_fast_group_512(proto, g, mode, kind, fp64, s);
        case 1024: return launch_fast_group_1024(proto, g, mode, kind, fp64, s);
        case 100: return launch_fast_group_100(proto, g, mode, kind, fp64, s);
        case 200: return launch_fast_group_200(proto, g, mode, kind, fp64, s);
        case 400: return launch_fast_group_400(proto, g, mode, kind, fp64, s);
        case 500: return launch_fast_group_500(proto, g, mode, kind, fp64, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace vg
