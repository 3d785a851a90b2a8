// Passes for power-of-two line lengths with the register-resident FFT.
// Same data layout and semantics as the LDS-staged passes of kernels.hpp;
// the host picks these whenever a line length is a power of two in
// [16, 4096].
#pragma once

#include "kernels.hpp"
#include "reg_fft.hpp"

namespace scfft {

// Block reduction of the five fp64 partial sums (wave64 shuffles, then LDS);
// quantity k goes to out[k * stride].
template <int NTH>
__device__ __forceinline__ void block_reduce5(Acc acc, double* red_lds, double* out, long long stride,
                                              int tid) {
  double v[5] = {acc.Jr, acc.Ji, acc.e2, acc.d2, acc.eJ};
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    double s = v[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    v[k] = s;
  }
  constexpr int NW = NTH / 64;
  const int lane = tid & 63, wave = tid >> 6;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 5; ++k) red_lds[k * NW + wave] = v[k];
  }
  __syncthreads();
  if (tid < 5) {
    double s = 0;
    for (int w = 0; w < NW; ++w) s += red_lds[tid * NW + w];
    out[tid * stride] = s;
  }
}

template <int N, int R>
struct XPassShape {
  static constexpr int TL = N / R;
  static constexpr int LINES = TL >= 256 ? 1 : 256 / TL;
  static constexpr int NTH = TL * LINES;
};

// x pass: LINES rows of one component per workgroup, TL threads per row;
// MK selects the local map at compile time.
template <typename T, int N, int R, int MK>
__global__ __launch_bounds__((XPassShape<N, R>::NTH)) void xpass_p2_kernel(XArgs a) {
  using SH = XPassShape<N, R>;
  constexpr int TL = SH::TL, LINES = SH::LINES, NTH = SH::NTH;
  constexpr int LP = P2Plan<N, R>::LP;
  const int solve = blockIdx.z;
  const int comp = blockIdx.y;
  if (!a.ignore_done && a.ctl[solve].done) return;
  extern __shared__ unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const int tid = threadIdx.x;
  const int line = tid / TL;
  const int j = tid - line * TL;
  const long long row = (long long)blockIdx.x * LINES + line;
  const bool valid = row < a.nlines;
  const long long fbase = ((long long)solve * a.d + comp) * a.M;
  const long long base = row * N;
  cx<T>* X = reinterpret_cast<cx<T>*>(a.X) + fbase + base;
  const cx<T>* tw = reinterpret_cast<const cx<T>*>(a.tw);
  cx<T> v[R];
#pragma unroll
  for (int i = 0; i < R; ++i) v[i] = valid ? X[j + TL * i] : mk<T>(0, 0);
  LocalMap<T, MK> lm;
  lm.load(a, solve, comp, fbase);
  // the phase map and E_prev do not depend on the FFT: load them first
  constexpr bool PF = MK == MAP_LIN || MK == MAP_ACC_EM || MK == MAP_ACC_MS;
  bool ph[R];
  cx<T> epo[R];
  if (PF && valid) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const long long g = base + j + TL * i;
      ph[i] = lm.phase[g] != 0;
      epo[i] = lm.Ep[g];
    }
  }
  cx<T>* slot = lds + line * LP;
  reg_fft<T, N, R>(v, slot, j, (T)1, tw);
  Acc acc;
  if (valid) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const long long g = base + j + TL * i;
      v[i] = PF ? lm.apply_pf(v[i], g, ph[i], epo[i], acc) : lm.apply(v[i], g, acc);
      acc_settle<true>(acc);
    }
  }
  reg_fft<T, N, R>(v, slot, j, (T)-1, tw);
  if (valid) {
#pragma unroll
    for (int i = 0; i < R; ++i) X[j + TL * i] = v[i];
  }
  __syncthreads();   // the FFT slots are free again
  block_reduce5<NTH>(acc, reinterpret_cast<double*>(smem_raw),
                     a.part + ((long long)solve * a.d + comp) * 5 * gridDim.x + blockIdx.x,
                     gridDim.x, tid);
}

// Lines per workgroup of the strided passes.  Every line keeps D LDS slots
// (its D components are transformed together); the tile is the widest power
// of two (at most 8 lines, 512 threads) whose slots fit the LDS budget,
// preferring the padded slot layout; narrower tiles (CW) are the autotuner's
// other candidates.
constexpr int kLineLdsBudget = 81920;

template <typename T, int N, int R, int D, int CW = 0>
struct LineShape {
  static constexpr int TL = N / R;
  static constexpr int PB = P2Plan<N, R>::LP * (int)sizeof(cx<T>) * D;   // padded bytes per line
  static constexpr int UB = N * (int)sizeof(cx<T>) * D;                  // unpadded
  static constexpr int CT = 512 / TL > 0 ? (512 / TL > 8 ? 8 : 512 / TL) : 1;
  static constexpr int CU = kLineLdsBudget / UB;                         // fits unpadded
  static constexpr int CF = CU >= 8 ? 8 : CU >= 4 ? 4 : CU >= 2 ? 2 : 1;
  static constexpr int CM = CF < CT ? CF : CT;
  static constexpr int CP = (CW > 0 && CW < CM) ? CW : CM;
  static constexpr int C = (CP * PB <= kLineLdsBudget || CP == 1) ? CP
                         : (CP / 2 * PB <= kLineLdsBudget || CP == 2) ? CP / 2
                         : (CP / 4 * PB <= kLineLdsBudget || CP == 4) ? CP / 4 : CP / 8;
  static constexpr bool PAD = C * PB <= kLineLdsBudget;
  static constexpr int LP = PAD ? P2Plan<N, R>::LP : N;
  static constexpr int NTH = TL * C;
  // adjacent columns' slots start 8 elements off a 64-bank boundary, so the
  // two columns a wave's lanes interleave do not hit the same banks
  // (measured: fp32 1-2 component lines faster, 3-component lines slower)
  static constexpr int CPAD = (sizeof(T) == 4 && C > 1 && D < 3) ? 8 : 0;
  static constexpr int CS = D * LP + CPAD;
  static constexpr int LDS = C * CS * (int)sizeof(cx<T>);
};

// The two per-axis symbol-table entries of mode m (see symbol_table_kernel).
template <typename T, int D>
__device__ __forceinline__ void symbol_entries(const GArgs& a, const int* m, T (*tv)[2]) {
#pragma unroll
  for (int q = 0; q < D; ++q) {
    const double* t = a.symtab[q] + 2 * m[q];
    tv[q][0] = (T)t[0];
    tv[q][1] = (T)t[1];
  }
}

// Symbol vector of eq. J11 on the grid for one mode from its table entries.
template <typename T, int D>
__device__ __forceinline__ T mode_symbol_t(int symbol, const T (*tv)[2], cx<T>* nv) {
  if (symbol == SYM_ROTATED) {
    T s[D], c[D];
#pragma unroll
    for (int q = 0; q < D; ++q) {
      s[q] = tv[q][0];
      c[q] = tv[q][1];
    }
    T nrm = 0;
#pragma unroll
    for (int q = 0; q < D; ++q) {
      T v = s[q];
#pragma unroll
      for (int l = 0; l < D; ++l)
        if (l != q) v *= c[l];
      nv[q] = mk<T>(v, 0);
      nrm += v * v;
    }
    if (nrm == (T)0) {
      // n = 0 at m != 0 (two or more Nyquist indices): the Nyquist-indicator
      // direction, scaled per axis (s[q] = n_q at a Nyquist index)
#pragma unroll
      for (int q = 0; q < D; ++q) {
        const T v = (c[q] == (T)0) ? s[q] : (T)0;
        nv[q] = mk<T>(v, 0);
        nrm += v * v;
      }
    }
    return nrm;
  } else if (symbol == SYM_SPECTRAL) {
    T v[D];
    bool nyq[D];
    bool has_nyq = false, has_other = false;
#pragma unroll
    for (int q = 0; q < D; ++q) {
      v[q] = tv[q][0];
      nyq[q] = tv[q][1] != (T)0;
      has_nyq |= nyq[q];
      has_other |= (!nyq[q]) && (v[q] != (T)0);
    }
    T nrm = 0;
#pragma unroll
    for (int q = 0; q < D; ++q) {
      const T w = (has_nyq && has_other && nyq[q]) ? (T)0 : v[q];
      nv[q] = mk<T>(w, 0);
      nrm += w * w;
    }
    return nrm;
  } else {
    T nrm = 0;
#pragma unroll
    for (int q = 0; q < D; ++q) {
      nv[q] = mk<T>(tv[q][0], tv[q][1]);
      nrm += norm2(nv[q]);
    }
    return nrm;
  }
}

// Gamma_1 step of eq. J11 (J44-J45 in H'') at one Fourier mode m for the D
// components w: at k = 0 the scheme's source term, elsewhere
// w <- ga w + gb n (n . w) / |n|^2 with the symbol vector n of the mode.
template <typename T, int D>
__device__ __forceinline__ void gamma_mode(const GArgs& a, const SolveCoef& cf, T ga, T gb, T keep,
                                           const int* m, const T (*tv)[2], cx<T>* w) {
  const bool zero = (m[0] == 0) && (m[1] == 0) && (D == 2 || m[2] == 0);
  if (zero) {
#pragma unroll
    for (int cc = 0; cc < D; ++cc) w[cc] = keep * w[cc] + ld2<T>(cf.kz_src[cc]);
    return;
  }
  cx<T> nv[3];
  const T nrm = mode_symbol_t<T, D>(a.symbol, tv, nv);
  cx<T> dot = mk<T>(0, 0);
  if (a.symbol == SYM_NETWORK) {
#pragma unroll
    for (int cc = 0; cc < D; ++cc) dot = dot + conj(nv[cc]) * w[cc];
  } else {
#pragma unroll
    for (int cc = 0; cc < D; ++cc) dot = dot + nv[cc] * w[cc];
  }
  const T inv = (T)1 / nrm;
#pragma unroll
  for (int cc = 0; cc < D; ++cc) w[cc] = ga * w[cc] + gb * (inv * (nv[cc] * dot));
}

// Strided passes: a tile of C lines adjacent along x, thread (j, c) with c
// fastest so that each row of the tile is one contiguous segment.
//   mode 0: forward FFT, Gamma_1 (eq. J11 / J44-J45) with the scheme's k = 0
//           source, inverse FFT -- all D = d components of one solve;
//   mode 1 / 2: forward / inverse FFT only (3D y pass), D = 1 component.
// Tiles are ordered so that consecutive tiles run on the same XCD (the
// hardware deals workgroups round-robin over the 8 XCDs), letting one L2
// serve the neighbouring row segments of adjacent tiles.
template <typename T, int N, int R, int D, int CW>
__global__ __launch_bounds__((LineShape<T, N, R, D, CW>::NTH)) void line_p2_kernel(GArgs a) {
  using SH = LineShape<T, N, R, D, CW>;
  constexpr int TL = SH::TL, C = SH::C, LP = SH::LP;
  const bool gam = (a.mode == 0);
  const int d = a.d;
  const int solve = gam ? blockIdx.z : blockIdx.z / d;
  const int comp0 = gam ? 0 : blockIdx.z % d;
  // done was set by an earlier kernel (or, harmlessly, by this one's
  // finalizing workgroup: a stale read only costs a wasted tile)
  if (!a.ignore_done && a.ctl[solve].done) return;
  extern __shared__ unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const int tid = threadIdx.x;
  // The Gamma pass also reduces the x pass's partials and applies the stop
  // rules: the grid then has one extra column of workgroups, and the
  // one at y = 0 of each solve does only that, beside the FFT tiles rather
  // than in front of one of them (in a grid of one row it is dispatched
  // last, so it does not hold a CU slot that a tile needs).
  const int nbx = gridDim.x - (a.fin ? 1 : 0), nby = gridDim.y;
  if (a.fin && (int)blockIdx.x == nbx) {
    if (blockIdx.y == 0 && comp0 == 0) finalize_solve(a.f, solve, tid, SH::NTH);
    return;
  }
  const int bxi = (int)blockIdx.x;
  const int c = tid % C;
  const int j = tid / C;
  // XCD-aware tile order
  const int nb = nbx * nby;
  const int b = blockIdx.y * nbx + bxi;
  int t = b;
  const int full = nb - nb % 8;
  if (b < full) t = (b % 8) * (full / 8) + b / 8;
  const int bx = t % nbx, by = t / nbx;
  const int x0 = bx * C;
  const bool valid = x0 + c < a.n[0];
  // uniform 64-bit tile base + 32-bit per-lane element offsets
  const long long M = a.M;
  cx<T>* X = reinterpret_cast<cx<T>*>(a.X) + ((long long)solve * d + comp0) * M + x0 +
             (long long)by * a.rp * (gam ? 1 : a.n[1]);
  const unsigned int Mu = (unsigned int)M, su = (unsigned int)a.stride;
  const unsigned int lane_off = (unsigned int)c + (unsigned int)j * su;
  const cx<T>* tw = reinterpret_cast<const cx<T>*>(a.tw);
  cx<T> v[D][R];
#pragma unroll
  for (int cc = 0; cc < D; ++cc)
#pragma unroll
    for (int i = 0; i < R; ++i)
      v[cc][i] = valid ? X[cc * Mu + lane_off + (unsigned int)(TL * i) * su] : mk<T>(0, 0);
  cx<T>* slot = lds + c * SH::CS;
  // symbol-table entries of this thread's modes: loaded before the FFT so
  // their latency hides under it
  T tab[R][D][2];
  if (gam && valid) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      int m[3];
      m[0] = x0 + c;
      if (D == 2) {
        m[1] = j + TL * i;
      } else {
        m[1] = by;
        m[2] = j + TL * i;
      }
      symbol_entries<T, D>(a, m, tab[i]);
    }
  }
  if (a.mode != 2) reg_fft_multi<T, N, R, SH::PAD, D>(v, slot, LP, j, (T)-1, tw);
  // 2D real mode: column 0 of tile 0 carries kx = 0 in its real and
  // kx = n0/2 in its imaginary part, both real along y, so after the y-FFT
  //   Z(k) = A(k) + i B(k),  A = (Z(k) + conj Z(-k)) / 2,  B = (Z(k) - conj Z(-k)) / 2i;
  // the mirrored values come through the column's LDS slot.
  const bool pk = gam && a.packed && x0 == 0;   // uniform over the workgroup
  if (pk) {
    __syncthreads();   // the forward FFT's last LDS reads are done
    if (c == 0) {
#pragma unroll
      for (int cc = 0; cc < D; ++cc)
#pragma unroll
        for (int i = 0; i < R; ++i) slot[cc * LP + lpad<SH::PAD>(j + TL * i)] = v[cc][i];
    }
    __syncthreads();
  }
  if (gam && valid) {
    const SolveCoef& cf = a.coef[solve];
    const T ga = (T)cf.ga, gb = (T)cf.gb, keep = (T)cf.kz_keep;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      int m[3];
      m[0] = x0 + c;
      if (D == 2) {
        m[1] = j + TL * i;
      } else {
        m[1] = by;
        m[2] = j + TL * i;
      }
      cx<T> w[D];
#pragma unroll
      for (int cc = 0; cc < D; ++cc) w[cc] = v[cc][i];
      // (a branch per mode keeps the registers of one mode live at a time)
      if (D == 2 && pk && c == 0) {
        const int km = (N - (j + TL * i)) & (N - 1);
        cx<T> b[D];
#pragma unroll
        for (int cc = 0; cc < D; ++cc) {
          const cx<T> zm = conj(slot[cc * LP + lpad<SH::PAD>(km)]);
          const cx<T> s = w[cc] + zm, df = w[cc] - zm;
          w[cc] = mk<T>((T)0.5 * s.x, (T)0.5 * s.y);
          b[cc] = mk<T>((T)0.5 * df.y, (T)-0.5 * df.x);
        }
        const int mn[3] = {a.n[0], m[1], 0};   // kx = n0/2 (= the column count)
        T tn[D][2];
        symbol_entries<T, D>(a, mn, tn);
        gamma_mode<T, D>(a, cf, ga, gb, keep, m, tab[i], w);
        gamma_mode<T, D>(a, cf, ga, gb, keep, mn, tn, b);
#pragma unroll
        for (int cc = 0; cc < D; ++cc) v[cc][i] = mk<T>(w[cc].x - b[cc].y, w[cc].y + b[cc].x);
      } else {
        gamma_mode<T, D>(a, cf, ga, gb, keep, m, tab[i], w);
#pragma unroll
        for (int cc = 0; cc < D; ++cc) v[cc][i] = w[cc];
      }
    }
  }
  if (a.mode != 1) reg_fft_multi<T, N, R, SH::PAD, D>(v, slot, LP, j, (T)1, tw);
  if (valid) {
#pragma unroll
    for (int cc = 0; cc < D; ++cc)
#pragma unroll
      for (int i = 0; i < R; ++i) X[cc * Mu + lane_off + (unsigned int)(TL * i) * su] = v[cc][i];
  }
}

}  // namespace scfft
