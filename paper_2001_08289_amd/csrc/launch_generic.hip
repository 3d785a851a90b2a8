// Instantiations of the LDS-staged mixed-radix passes (any 2/3/5-smooth
// line length) for both precisions.
#include "launch.hpp"

namespace scfft {
namespace {
constexpr int kNT = 1024;
// elements a workgroup transforms at once (64 KiB of LDS in both precisions)
template <typename T>
constexpr int emax() { return (sizeof(T) == 4 ? 8192 : 4096) / kNT; }
}  // namespace

template <typename T>
void launch_xpass_generic(const XArgs& a, dim3 grid, size_t lds, hipStream_t st) {
  hipLaunchKernelGGL((xpass_kernel<T, kNT, emax<T>()>), grid, dim3(kNT), lds, st, a);
}

template <typename T>
void launch_line_generic(const GArgs& a, dim3 grid, size_t lds, hipStream_t st) {
  hipLaunchKernelGGL((line_pass_kernel<T, kNT, emax<T>()>), grid, dim3(kNT), lds, st, a);
}

// Radix 16 (2048 = 16*8*16, one LDS exchange fewer) measured faster only for
// the fp64 Gamma pass of 2048^2 grids (115 -> 104 us).
void launch_line_r16_f64_2048(const GArgs& a, dim3 grid, hipStream_t st) {
  using SH = LineShape<double, 2048, 16, 2, 0>;
  const size_t lds = (size_t)SH::LDS;
  if (lds > 65536) {
    static bool set = false;
    if (!set) {
      (void)hipFuncSetAttribute((const void*)line_p2_kernel<double, 2048, 16, 2, 0>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      set = true;
    }
  }
  hipLaunchKernelGGL((line_p2_kernel<double, 2048, 16, 2, 0>), grid, dim3(SH::NTH), lds, st, a);
}

template void launch_xpass_generic<float>(const XArgs&, dim3, size_t, hipStream_t);
template void launch_xpass_generic<double>(const XArgs&, dim3, size_t, hipStream_t);
template void launch_line_generic<float>(const GArgs&, dim3, size_t, hipStream_t);
template void launch_line_generic<double>(const GArgs&, dim3, size_t, hipStream_t);

}  // namespace scfft
