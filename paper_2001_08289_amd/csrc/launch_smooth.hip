// Instantiations of the compile-time mixed-radix passes for one precision
// (SCFFT_T) and one kernel family (SCFFT_SMK: 0..3 the x pass of a
// full-complex field with that local map; 4 / 5 the Gamma pass of a 2D / 3D
// grid; 6 the 3D y pass; 7..10 the real-field x pass with local map
// SCFFT_SMK - 7), both set by the build.
#include "launch.hpp"

#if !defined(SCFFT_T) || !defined(SCFFT_SMK)
#error "SCFFT_T (float or double) and SCFFT_SMK (0..10) must be defined"
#endif

namespace scfft {
namespace {

template <typename T, int N>
bool smooth_sm(const XArgs& xa, const GArgs& ga, dim3 grid, hipStream_t st) {
  using SH = SmShape<T, N>;
  static_assert(SH::XLDS <= 65536, "x-pass workgroup LDS within 64 KiB");
  if constexpr (SCFFT_SMK >= 7) {
    (void)ga;
    hipLaunchKernelGGL((xpass_sm_r2c_kernel<T, N, SCFFT_SMK - 7>), grid, dim3(64 * SH::XW),
                       (size_t)SH::XLDS, st, xa);
  } else if constexpr (SCFFT_SMK >= 4) {
    (void)xa;
    constexpr int D = SCFFT_SMK == 4 ? 2 : SCFFT_SMK == 5 ? 3 : 1;
    using TS = SmTile<T, N, D>;
    static_assert(TS::LDS <= 160 * 1024, "workgroup LDS within gfx950's 160 KiB");
    if (TS::LDS > 65536) {
      // LDS beyond 64 KiB per workgroup is opt-in
      static bool set = false;
      if (!set) {
        (void)hipFuncSetAttribute((const void*)line_sm_kernel<T, N, D>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)TS::LDS);
        set = true;
      }
    }
    hipLaunchKernelGGL((line_sm_kernel<T, N, D>), grid, dim3(TS::NT), (size_t)TS::LDS, st, ga);
  } else {
    (void)ga;
    hipLaunchKernelGGL((xpass_sm_kernel<T, N, SCFFT_SMK>), grid, dim3(64 * SH::XW),
                       (size_t)SH::XLDS, st, xa);
  }
  return true;
}

}  // namespace

template <>
bool launch_smooth_unit<SCFFT_T, SCFFT_SMK>(const XArgs* xa, const GArgs* ga, dim3 grid,
                                            hipStream_t st, int n) {
  static const XArgs x0{};
  static const GArgs g0{};
  const XArgs& x = xa ? *xa : x0;
  const GArgs& g = ga ? *ga : g0;
#define C_(N) return smooth_sm<SCFFT_T, N>(x, g, grid, st)
  SCFFT_SMOOTH_SWITCH(n, C_)
#undef C_
  return false;
}

}  // namespace scfft
