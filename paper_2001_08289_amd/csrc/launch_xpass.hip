// Instantiations of the register-resident x passes (real-field and complex)
// for one precision, SCFFT_T (float or double), set by the build.
#include "launch.hpp"

#ifndef SCFFT_T
#error "SCFFT_T must name the field precision (float or double)"
#endif

namespace scfft {
namespace {

template <typename T, int N, bool NT, int RR>
void xreal_t(const XArgs& a, dim3 grid, hipStream_t st, int mk) {
  using SH = XPassShape<N, RR>;
  const size_t lds = std::max((size_t)SH::LINES * P2Plan<N, RR>::LP * sizeof(cx<T>),
                              (size_t)5 * (SH::NTH / 64) * sizeof(double));
  switch (mk) {
    case MAP_LIN:
      hipLaunchKernelGGL((xpass_r2c_kernel<T, N, RR, MAP_LIN, NT>), grid, dim3(SH::NTH), lds, st, a);
      break;
    case MAP_LIN_DENS:
      hipLaunchKernelGGL((xpass_r2c_kernel<T, N, RR, MAP_LIN_DENS, NT>), grid, dim3(SH::NTH), lds, st, a);
      break;
    case MAP_ACC_EM:
      hipLaunchKernelGGL((xpass_r2c_kernel<T, N, RR, MAP_ACC_EM, NT>), grid, dim3(SH::NTH), lds, st, a);
      break;
    default:
      hipLaunchKernelGGL((xpass_r2c_kernel<T, N, RR, MAP_ACC_MS, NT>), grid, dim3(SH::NTH), lds, st, a);
      break;
  }
}

template <typename T, int N, int RR>
void xreg_t(const XArgs& a, dim3 grid, hipStream_t st, int mk) {
  using SH = XPassShape<N, RR>;
  const size_t lds = std::max((size_t)SH::LINES * P2Plan<N, RR>::LP * sizeof(cx<T>),
                              (size_t)5 * (SH::NTH / 64) * sizeof(double));
  switch (mk) {
    case MAP_LIN:
      hipLaunchKernelGGL((xpass_p2_kernel<T, N, RR, MAP_LIN>), grid, dim3(SH::NTH), lds, st, a);
      break;
    case MAP_LIN_DENS:
      hipLaunchKernelGGL((xpass_p2_kernel<T, N, RR, MAP_LIN_DENS>), grid, dim3(SH::NTH), lds, st, a);
      break;
    case MAP_ACC_EM:
      hipLaunchKernelGGL((xpass_p2_kernel<T, N, RR, MAP_ACC_EM>), grid, dim3(SH::NTH), lds, st, a);
      break;
    default:
      hipLaunchKernelGGL((xpass_p2_kernel<T, N, RR, MAP_ACC_MS>), grid, dim3(SH::NTH), lds, st, a);
      break;
  }
}

}  // namespace

template <>
void launch_xpass_real<SCFFT_T>(const XArgs& a, dim3 grid, hipStream_t st, int n0, int mk, bool nt,
                                int xr) {
  if (nt) {
    if (xr == 8) {
#define C_(N) xreal_t<SCFFT_T, N, true, 8>(a, grid, st, mk)
      SCFFT_P2_SWITCH(n0, C_)
#undef C_
    } else {
#define C_(N) xreal_t<SCFFT_T, N, true, 4>(a, grid, st, mk)
      SCFFT_P2_SWITCH(n0, C_)
#undef C_
    }
  } else {
    if (xr == 8) {
#define C_(N) xreal_t<SCFFT_T, N, false, 8>(a, grid, st, mk)
      SCFFT_P2_SWITCH(n0, C_)
#undef C_
    } else {
#define C_(N) xreal_t<SCFFT_T, N, false, 4>(a, grid, st, mk)
      SCFFT_P2_SWITCH(n0, C_)
#undef C_
    }
  }
}

template <>
void launch_xpass_reg<SCFFT_T>(const XArgs& a, dim3 grid, hipStream_t st, int n0, int mk, int xr) {
  if (xr == 8) {
#define C_(N) xreg_t<SCFFT_T, N, 8>(a, grid, st, mk)
    SCFFT_P2_SWITCH(n0, C_)
#undef C_
  } else {
#define C_(N) xreg_t<SCFFT_T, N, 4>(a, grid, st, mk)
    SCFFT_P2_SWITCH(n0, C_)
#undef C_
  }
}

}  // namespace scfft
