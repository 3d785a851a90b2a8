// Instantiations of the register-resident strided passes for one precision
// (SCFFT_T) and one component count (SCFFT_D: 1 = plain 3D y pass, 2 / 3 =
// Gamma pass of a 2D / 3D grid), both set by the build.
#include "launch.hpp"

#if !defined(SCFFT_T) || !defined(SCFFT_D)
#error "SCFFT_T (float or double) and SCFFT_D (1, 2 or 3) must be defined"
#endif

namespace scfft {
namespace {

template <typename T, int N, int D, int CW, int RR>
void line_cw(const GArgs& a, dim3 grid, hipStream_t st) {
  using SH = LineShape<T, N, RR, D, CW>;
  const size_t lds = (size_t)SH::LDS;
  if (lds > 65536) {
    // LDS beyond 64 KiB per workgroup (gfx950 has 160 KiB per CU) is opt-in
    static bool set = false;
    if (!set) {
      (void)hipFuncSetAttribute((const void*)line_p2_kernel<T, N, RR, D, CW>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      set = true;
    }
  }
  hipLaunchKernelGGL((line_p2_kernel<T, N, RR, D, CW>), grid, dim3(SH::NTH), lds, st, a);
}

template <typename T, int N, int D, int RR>
void line_n(const GArgs& a, dim3 grid, hipStream_t st) {
  if constexpr ((D == 3 && N > 1024) || N < RR) {
    return;   // 3D Gamma lines are at most 1024 points (host limit)
  } else {
    switch (a.C) {
      case 1: line_cw<T, N, D, 1, RR>(a, grid, st); break;
      case 2: line_cw<T, N, D, 2, RR>(a, grid, st); break;
      case 4: line_cw<T, N, D, 4, RR>(a, grid, st); break;
      case 8: line_cw<T, N, D, 8, RR>(a, grid, st); break;
      default: line_cw<T, N, D, 0, RR>(a, grid, st); break;
    }
  }
}

}  // namespace

template <>
void launch_line_reg<SCFFT_T, SCFFT_D>(const GArgs& a, dim3 grid, hipStream_t st, int n, int gr) {
  // the Gamma passes offer radix 4 and 8; the plain 3D y pass radix 8
  if (SCFFT_D != 1 && gr == 4) {
#define C_(N) line_n<SCFFT_T, N, SCFFT_D, 4>(a, grid, st)
    SCFFT_P2_SWITCH(n, C_)
#undef C_
  } else {
#define C_(N) line_n<SCFFT_T, N, SCFFT_D, 8>(a, grid, st)
    SCFFT_P2_SWITCH(n, C_)
#undef C_
  }
}

}  // namespace scfft
