// Instantiations of the compile-time mixed-radix passes for one precision
// (SCFFT_T, set by the build).
#include "launch.hpp"

#if !defined(SCFFT_T)
#error "SCFFT_T (float or double) must be defined"
#endif

namespace scfft {
namespace {

template <typename T, int N>
bool xpass_sm(const XArgs& a, dim3 grid, hipStream_t st) {
  constexpr size_t lds = (size_t)sm_lines<T, N>() * N * sizeof(cx<T>);
  static_assert(lds >= 5 * (kSmNT / 64) * sizeof(double), "reduction must fit the LDS");
  hipLaunchKernelGGL((xpass_sm_kernel<T, N>), grid, dim3(kSmNT), lds, st, a);
  return true;
}

template <typename T, int N>
bool gamma_sm(const GArgs& a, dim3 grid, hipStream_t st) {
  constexpr size_t lds = (size_t)2 * sm_cols<T, N>() * N * sizeof(cx<T>);
  hipLaunchKernelGGL((gamma_sm_kernel<T, N>), grid, dim3(kSmNT), lds, st, a);
  return true;
}

}  // namespace

template <>
bool launch_xpass_smooth<SCFFT_T>(const XArgs& a, dim3 grid, hipStream_t st, int n) {
#define C_(N) return xpass_sm<SCFFT_T, N>(a, grid, st)
  SCFFT_SMOOTH_SWITCH(n, C_)
#undef C_
  return false;
}

template <>
bool launch_gamma_smooth<SCFFT_T>(const GArgs& a, dim3 grid, hipStream_t st, int n) {
#define C_(N) return gamma_sm<SCFFT_T, N>(a, grid, st)
  SCFFT_SMOOTH_SWITCH(n, C_)
#undef C_
  return false;
}

}  // namespace scfft
