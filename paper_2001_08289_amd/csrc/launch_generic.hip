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

int xpass_lines(int n, int esz, int xr) {
  int r = 1;
  if (xr == 8) {
#define C_(N) r = XPassShape<N, 8>::LINES
    SCFFT_P2_SWITCH(n, C_)
#undef C_
  } else {
#define C_(N) r = XPassShape<N, 4>::LINES
    SCFFT_P2_SWITCH(n, C_)
#undef C_
  }
  (void)esz;
  return r;
}

namespace {
template <typename T, int D, int RR>
int tile_max_t(int n) {
  int r = 1;
#define C_(N) r = (N >= RR) ? LineShape<T, N, (N >= RR ? RR : N), D>::C : 1
  SCFFT_P2_SWITCH(n, C_)
#undef C_
  return r;
}
template <typename T>
int tile_max_r(int n, int D, int gr) {
  if (gr == 16) return D == 2 ? tile_max_t<T, 2, 16>(n) : 1;
  if (gr == 4) return D == 1 ? tile_max_t<T, 1, 4>(n) : D == 2 ? tile_max_t<T, 2, 4>(n) : tile_max_t<T, 3, 4>(n);
  return D == 1 ? tile_max_t<T, 1, 8>(n) : D == 2 ? tile_max_t<T, 2, 8>(n) : tile_max_t<T, 3, 8>(n);
}
}  // namespace

int line_tile_max(int n, int esz, int D, int gr) {
  return esz == 8 ? tile_max_r<float>(n, D, gr) : tile_max_r<double>(n, D, gr);
}

int smooth_lines(int n, int esz) {
  if (esz == 8) {
#define C_(N) return SmShape<float, N>::XL
    SCFFT_SMOOTH_SWITCH(n, C_)
#undef C_
  } else {
#define C_(N) return SmShape<double, N>::XL
    SCFFT_SMOOTH_SWITCH(n, C_)
#undef C_
  }
  return 0;
}

int smooth_cols(int n, int esz, int D) {
  if (esz == 8) {
#define C_(N) return D == 2 ? SmTile<float, N, 2>::C : D == 3 ? SmTile<float, N, 3>::C : SmTile<float, N, 1>::C
    SCFFT_SMOOTH_SWITCH(n, C_)
#undef C_
  } else {
#define C_(N) return D == 2 ? SmTile<double, N, 2>::C : D == 3 ? SmTile<double, N, 3>::C : SmTile<double, N, 1>::C
    SCFFT_SMOOTH_SWITCH(n, C_)
#undef C_
  }
  return 0;
}

template void launch_xpass_generic<float>(const XArgs&, dim3, size_t, hipStream_t);
template void launch_xpass_generic<double>(const XArgs&, dim3, size_t, hipStream_t);
template void launch_line_generic<float>(const GArgs&, dim3, size_t, hipStream_t);
template void launch_line_generic<double>(const GArgs&, dim3, size_t, hipStream_t);

}  // namespace scfft
