// Register-resident Stockham FFT for power-of-two line lengths (gfx950).
//
// A line of N points is owned by TL = N/R threads; thread j holds elements
// j + TL*i (i = 0..R-1) in registers before and after the transform, so a
// pointwise real-space update can sit between an inverse and a forward FFT
// without touching memory.  Passes have radix R except one remainder pass
// (R = 8: 2048 = 8*4*8*8); every radix divides R, so each thread owns R/r
// butterflies per pass.  The first pass reads registers, the last pass writes
// registers, and the exchanges between passes go through an LDS slot of
// N + N/16 elements (one pad element per 16 spreads the strided writes over
// the banks).  All index arithmetic is compile time except the lane index.
#pragma once

#include "device_fft.hpp"

namespace scfft {

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }

template <int N, int R>
struct P2Plan {
  static constexpr int TL = N / R;
  static constexpr int LN = ilog2(N);
  static constexpr int LR = ilog2(R);
  static constexpr int NFULL = LN / LR;
  static constexpr int REM = 1 << (LN - NFULL * LR);
  static constexpr int NPASS = NFULL + (REM > 1 ? 1 : 0);
  // the remainder radix runs as the second pass (or the only second pass)
  static constexpr int radix(int p) { return (REM > 1 && p == 1) ? REM : R; }
  static constexpr int LP = N + N / 16;  // padded LDS slot length
  static_assert((1 << LN) == N && (1 << LR) == R && N >= R, "power-of-two sizes only");
};

template <bool PAD>
__device__ __forceinline__ int lpad(int i) { return PAD ? i + (i >> 4) : i; }

template <typename T, int N, int R, int P, int NS, bool PAD>
struct P2Pass {
  using PL = P2Plan<N, R>;
  static constexpr int r = PL::radix(P);
  static constexpr int NB = R / r;            // butterflies per thread
  static constexpr int TL = PL::TL;
  static constexpr bool FIRST = (P == 0);
  static constexpr bool LAST = (NS * r == N);
  static constexpr int STEP = N / (NS * r);   // twiddle table stride

  __device__ __forceinline__ static void run(cx<T> (&v)[R], cx<T>* __restrict__ slot, int j, T sign,
                                             const cx<T>* __restrict__ tw) {
    cx<T> x[NB][r];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
#pragma unroll
      for (int q = 0; q < r; ++q) {
        if (FIRST) {
          x[u][q] = v[u + q * NB];
        } else {
          x[u][q] = slot[lpad<PAD>(j + u * TL + q * (N / r))];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int b = j + u * TL;
      if (NS > 1) {
        // one table load per butterfly; the powers w^q follow by products
        const int k = b & (NS - 1);
        cx<T> w1 = tw[k * STEP];
        if (sign > 0) w1.y = -w1.y;
        cx<T> wq[r];
        wq[1] = w1;
#pragma unroll
        for (int q = 2; q < r; ++q) wq[q] = (q & 1) ? wq[q - 1] * w1 : wq[q / 2] * wq[q / 2];
#pragma unroll
        for (int q = 1; q < r; ++q) x[u][q] = x[u][q] * wq[q];
      }
      Dft<T, r>::run(x[u], sign);
    }
    if (LAST) {
#pragma unroll
      for (int u = 0; u < NB; ++u)
#pragma unroll
        for (int q = 0; q < r; ++q) v[u + q * NB] = x[u][q];
    } else {
      __syncthreads();   // every thread has read this pass's inputs
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int b = j + u * TL;
        const int k = b & (NS - 1);
        const int idxd = (b / NS) * NS * r + k;
#pragma unroll
        for (int q = 0; q < r; ++q) slot[lpad<PAD>(idxd + q * NS)] = x[u][q];
      }
      __syncthreads();
      P2Pass<T, N, R, P + 1, NS * r, PAD>::run(v, slot, j, sign, tw);
    }
  }
};

// Terminal specialisation guard (never instantiated with NS >= N).
template <typename T, int N, int R, int P, bool PAD>
struct P2Pass<T, N, R, P, N, PAD> {
  __device__ __forceinline__ static void run(cx<T> (&)[R], cx<T>*, int, T, const cx<T>*) {}
};

// In-register FFT of one line; every thread of the workgroup must call it
// (it contains barriers).  slot: this line's LDS slot (P2Plan::LP elements
// with PAD, N without).
template <typename T, int N, int R, bool PAD = true>
__device__ __forceinline__ void reg_fft(cx<T> (&v)[R], cx<T>* __restrict__ slot, int j, T sign,
                                        const cx<T>* __restrict__ tw) {
  P2Pass<T, N, R, 0, 1, PAD>::run(v, slot, j, sign, tw);
}

template <typename T, int N, int R>
__device__ __forceinline__ void reg_fft_nopad(cx<T> (&v)[R], cx<T>* __restrict__ slot, int j, T sign,
                                              const cx<T>* __restrict__ tw) {
  P2Pass<T, N, R, 0, 1, false>::run(v, slot, j, sign, tw);
}

}  // namespace scfft

namespace scfft {

// D lines owned by the same threads, transformed together: each pass computes
// the twiddles once for all D lines and the D lines share the pass's two
// barriers.  Line dd uses the LDS slot at slot + dd*sstride.
template <typename T, int N, int R, int P, int NS, bool PAD, int D>
struct P2PassM {
  using PL = P2Plan<N, R>;
  static constexpr int r = PL::radix(P);
  static constexpr int NB = R / r;
  static constexpr int TL = PL::TL;
  static constexpr bool FIRST = (P == 0);
  static constexpr bool LAST = (NS * r == N);
  static constexpr int STEP = N / (NS * r);

  __device__ __forceinline__ static void run(cx<T> (&v)[D][R], cx<T>* __restrict__ slot,
                                             int sstride, int j, T sign,
                                             const cx<T>* __restrict__ tw) {
    cx<T> x[D][NB][r];
#pragma unroll
    for (int dd = 0; dd < D; ++dd)
#pragma unroll
      for (int u = 0; u < NB; ++u)
#pragma unroll
        for (int q = 0; q < r; ++q) {
          if (FIRST) {
            x[dd][u][q] = v[dd][u + q * NB];
          } else {
            x[dd][u][q] = slot[dd * sstride + lpad<PAD>(j + u * TL + q * (N / r))];
          }
        }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int b = j + u * TL;
      if (NS > 1) {
        const int k = b & (NS - 1);
        cx<T> w1 = tw[k * STEP];
        if (sign > 0) w1.y = -w1.y;
        cx<T> wq[r];
        wq[1] = w1;
#pragma unroll
        for (int q = 2; q < r; ++q) wq[q] = (q & 1) ? wq[q - 1] * w1 : wq[q / 2] * wq[q / 2];
#pragma unroll
        for (int dd = 0; dd < D; ++dd)
#pragma unroll
          for (int q = 1; q < r; ++q) x[dd][u][q] = x[dd][u][q] * wq[q];
      }
#pragma unroll
      for (int dd = 0; dd < D; ++dd) Dft<T, r>::run(x[dd][u], sign);
    }
    if (LAST) {
#pragma unroll
      for (int dd = 0; dd < D; ++dd)
#pragma unroll
        for (int u = 0; u < NB; ++u)
#pragma unroll
          for (int q = 0; q < r; ++q) v[dd][u + q * NB] = x[dd][u][q];
    } else {
      __syncthreads();
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int b = j + u * TL;
        const int k = b & (NS - 1);
        const int idxd = (b / NS) * NS * r + k;
#pragma unroll
        for (int dd = 0; dd < D; ++dd)
#pragma unroll
          for (int q = 0; q < r; ++q) slot[dd * sstride + lpad<PAD>(idxd + q * NS)] = x[dd][u][q];
      }
      __syncthreads();
      P2PassM<T, N, R, P + 1, NS * r, PAD, D>::run(v, slot, sstride, j, sign, tw);
    }
  }
};

template <typename T, int N, int R, int P, bool PAD, int D>
struct P2PassM<T, N, R, P, N, PAD, D> {
  __device__ __forceinline__ static void run(cx<T> (&)[D][R], cx<T>*, int, int, T, const cx<T>*) {}
};

template <typename T, int N, int R, bool PAD, int D>
__device__ __forceinline__ void reg_fft_multi(cx<T> (&v)[D][R], cx<T>* __restrict__ slot,
                                              int sstride, int j, T sign,
                                              const cx<T>* __restrict__ tw) {
  P2PassM<T, N, R, 0, 1, PAD, D>::run(v, slot, sstride, j, sign, tw);
}

}  // namespace scfft
