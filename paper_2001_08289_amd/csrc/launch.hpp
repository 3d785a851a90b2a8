// Launchers of the iteration passes.
//
// The kernels are templates over precision, line length, radix, tile width
// and local map; their instantiations are split over several translation
// units (launch_*.hip, each compiled once per precision) so that the library
// builds in parallel.  The host driver (scfft.hip) calls only the functions
// declared here.
#pragma once

#include "kernels_real.hpp"
#include "kernels_smooth.hpp"

namespace scfft {

#define SCFFT_P2_SWITCH(n, CALL)  \
  switch (n) {                    \
    case 16: CALL(16); break;     \
    case 32: CALL(32); break;     \
    case 64: CALL(64); break;     \
    case 128: CALL(128); break;   \
    case 256: CALL(256); break;   \
    case 512: CALL(512); break;   \
    case 1024: CALL(1024); break; \
    case 2048: CALL(2048); break; \
    case 4096: CALL(4096); break; \
    default: break;               \
  }

// Real-field x pass (power-of-two n0) with register radix xr (4 or 8):
// local map `mk`, own streams nontemporal when `nt`.  grid = (row-pair
// blocks, d, solves).
template <typename T>
void launch_xpass_real(const XArgs& a, dim3 grid, hipStream_t st, int n0, int mk, bool nt, int xr);

// Complex register-resident x pass (power-of-two n0), register radix xr.
template <typename T>
void launch_xpass_reg(const XArgs& a, dim3 grid, hipStream_t st, int n0, int mk, int xr);

// Register-resident strided pass over lines of length n: D = 2 / 3 the Gamma
// pass of a 2D / 3D grid (all components), D = 1 a plain 3D y pass; a.C is
// the tile width (one of 1, 2, 4, 8; anything else the widest that fits);
// gr the register radix (D = 2, 3: 4 or 8; D = 1: 8).
template <typename T, int D>
void launch_line_reg(const GArgs& a, dim3 grid, hipStream_t st, int n, int gr);

// Rows per workgroup of the register x pass and the widest strided tile,
// for a line length, precision (sizeof T), component count and radix.
int xpass_lines(int n, int esz, int xr);
int line_tile_max(int n, int esz, int D, int gr);

// fp64 Gamma pass of 2048-point columns with radix-16 register FFTs.
void launch_line_r16_f64_2048(const GArgs& a, dim3 grid, hipStream_t st);

// Line lengths with compile-time mixed-radix passes (full-complex x pass,
// Gamma pass, 3D y pass); every other 2/3/5-smooth length takes the
// runtime-planned passes below.
#define SCFFT_SMOOTH_SWITCH(n, CALL) \
  switch (n) {                       \
    case 48: CALL(48);               \
    case 80: CALL(80);               \
    case 90: CALL(90);               \
    case 96: CALL(96);               \
    case 120: CALL(120);             \
    case 160: CALL(160);             \
    case 180: CALL(180);             \
    case 192: CALL(192);             \
    case 240: CALL(240);             \
    case 288: CALL(288);             \
    case 320: CALL(320);             \
    case 360: CALL(360);             \
    case 384: CALL(384);             \
    case 400: CALL(400);             \
    case 432: CALL(432);             \
    case 480: CALL(480);             \
    case 576: CALL(576);             \
    case 640: CALL(640);             \
    case 720: CALL(720);             \
    case 768: CALL(768);             \
    case 800: CALL(800);             \
    case 864: CALL(864);             \
    case 900: CALL(900);             \
    case 960: CALL(960);             \
    default: break;                  \
  }

// Compile-time mixed-radix passes (one line per 64, 32 or 16 lanes): false
// (nothing launched) for a length without an instantiation.  x pass grid = (row
// blocks of smooth_lines rows, d, solves); Gamma grid = (column tiles of
// smooth_cols columns, 1 (2D) or n1 (3D), solves); 3D y pass grid = (column
// tiles, n2, solves x 3).
// mk: the x pass's local map (MapKind).  The real-field x pass (grid =
// (blocks of smooth_lines row pairs, d, solves)) takes no packed column.
template <typename T, int K>
bool launch_smooth_unit(const XArgs* xa, const GArgs* ga, dim3 grid, hipStream_t st, int n);
template <typename T>
bool launch_xpass_smooth(const XArgs& a, dim3 grid, hipStream_t st, int n, int mk) {
  switch (mk) {
    case MAP_LIN: return launch_smooth_unit<T, MAP_LIN>(&a, nullptr, grid, st, n);
    case MAP_LIN_DENS: return launch_smooth_unit<T, MAP_LIN_DENS>(&a, nullptr, grid, st, n);
    case MAP_ACC_EM: return launch_smooth_unit<T, MAP_ACC_EM>(&a, nullptr, grid, st, n);
    default: return launch_smooth_unit<T, MAP_ACC_MS>(&a, nullptr, grid, st, n);
  }
}
template <typename T>
bool launch_xpass_smooth_real(const XArgs& a, dim3 grid, hipStream_t st, int n, int mk) {
  switch (mk) {
    case MAP_LIN: return launch_smooth_unit<T, 7 + MAP_LIN>(&a, nullptr, grid, st, n);
    case MAP_LIN_DENS: return launch_smooth_unit<T, 7 + MAP_LIN_DENS>(&a, nullptr, grid, st, n);
    case MAP_ACC_EM: return launch_smooth_unit<T, 7 + MAP_ACC_EM>(&a, nullptr, grid, st, n);
    default: return launch_smooth_unit<T, 7 + MAP_ACC_MS>(&a, nullptr, grid, st, n);
  }
}
template <typename T>
bool launch_gamma_smooth(const GArgs& a, dim3 grid, hipStream_t st, int n, int d) {
  return d == 2 ? launch_smooth_unit<T, 4>(nullptr, &a, grid, st, n)
                : launch_smooth_unit<T, 5>(nullptr, &a, grid, st, n);
}
template <typename T>
bool launch_ypass_smooth(const GArgs& a, dim3 grid, hipStream_t st, int n) {
  return launch_smooth_unit<T, 6>(nullptr, &a, grid, st, n);
}
// Rows per x-pass workgroup; columns per strided tile for D components
// (2 / 3: Gamma pass, 1: 3D y pass).  0: no instantiation.
int smooth_lines(int n, int esz);
int smooth_cols(int n, int esz, int D);

// LDS-staged mixed-radix passes (any 2/3/5-smooth length).
template <typename T>
void launch_xpass_generic(const XArgs& a, dim3 grid, size_t lds, hipStream_t st);
template <typename T>
void launch_line_generic(const GArgs& a, dim3 grid, size_t lds, hipStream_t st);

}  // namespace scfft
