// Compile-time mixed-radix passes for 2/3/5-smooth line lengths (gfx950).
//
// The same LDS-staged Stockham transform as the runtime-planned passes of
// device_fft.hpp, but with the line length, the radix sequence, the lines per
// workgroup and the tile width fixed at compile time: every pass is unrolled,
// and the index arithmetic of the butterflies (divisions by the butterfly
// count, the stride and the tile width) folds into multiplications by
// constants instead of runtime integer divisions.  One instantiation per
// supported length (SCFFT_SMOOTH_SWITCH); other smooth lengths keep the
// runtime-planned passes.
#pragma once

#include "kernels_p2.hpp"

namespace scfft {

constexpr int kSmNT = 1024;   // threads per workgroup

// Elements one workgroup holds in LDS (64 KiB in both precisions).
template <typename T>
constexpr int sm_elems() { return sizeof(T) == 4 ? 8192 : 4096; }

// Radix of pass p for a length n: radix 8 while 8 divides, then one radix 4
// or 2 for the rest of the power of two, then the fives, then the threes;
// 0 once p is past the last pass.
constexpr int sm_radix(int n, int p) {
  int m = n, i = 0;
  while (m % 8 == 0) {
    if (i == p) return 8;
    m /= 8;
    ++i;
  }
  if (m % 4 == 0) {
    if (i == p) return 4;
    m /= 4;
    ++i;
  }
  if (m % 2 == 0) {
    if (i == p) return 2;
    m /= 2;
    ++i;
  }
  while (m % 5 == 0) {
    if (i == p) return 5;
    m /= 5;
    ++i;
  }
  while (m % 3 == 0) {
    if (i == p) return 3;
    m /= 3;
    ++i;
  }
  return 0;
}

// x pass: whole lines per workgroup; Gamma pass (2D): columns per tile.
template <typename T, int N>
constexpr int sm_lines() { return sm_elems<T>() / N; }
template <typename T, int N>
constexpr int sm_cols() {
  return sm_elems<T>() / (2 * N) > 16 ? 16 : sm_elems<T>() / (2 * N);
}

// One radix-r pass (stride NS) over NL lines of N points in LDS; line l's
// element k sits at l*LS + k*ES.  LF: consecutive butterflies walk the lines
// first (the strided tile layout), else the points of one line first.
template <typename T, int N, int NL, bool LF, int P, int NS>
__device__ __forceinline__ void sm_pass(cx<T>* __restrict__ lds, const cx<T>* __restrict__ tw,
                                        T sign, int tid) {
  if constexpr (NS < N) {
    constexpr int r = sm_radix(N, P);
    static_assert(r > 0 && N % (NS * r) == 0, "radix sequence must factor N");
    constexpr int NBL = N / r;          // butterflies per line
    constexpr int NB = NL * NBL;        // butterflies per workgroup
    constexpr int BPT = (NB + kSmNT - 1) / kSmNT;
    constexpr int STEP = N / (NS * r);  // twiddle table stride
    constexpr int LS = LF ? 1 : N;
    constexpr int ES = LF ? NL : 1;
    cx<T> v[BPT][r];
#pragma unroll
    for (int u = 0; u < BPT; ++u) {
      const int b = tid + u * kSmNT;
      if (NB % kSmNT == 0 || b < NB) {
        const int l = LF ? b % NL : b / NBL;
        const int j = LF ? b / NL : b - (b / NBL) * NBL;
        const cx<T>* base = lds + l * LS;
#pragma unroll
        for (int q = 0; q < r; ++q) v[u][q] = base[(j + q * NBL) * ES];
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < BPT; ++u) {
      const int b = tid + u * kSmNT;
      if (NB % kSmNT == 0 || b < NB) {
        const int l = LF ? b % NL : b / NBL;
        const int j = LF ? b / NL : b - (b / NBL) * NBL;
        const int k = j % NS;
        if constexpr (NS > 1) {
          // one table load per butterfly; the powers w^q follow by products
          cx<T> w1 = tw[k * STEP];
          if (sign > 0) w1.y = -w1.y;
          cx<T> wq[r];
          wq[1] = w1;
#pragma unroll
          for (int q = 2; q < r; ++q) wq[q] = (q & 1) ? wq[q - 1] * w1 : wq[q / 2] * wq[q / 2];
#pragma unroll
          for (int q = 1; q < r; ++q) v[u][q] = v[u][q] * wq[q];
        }
        Dft<T, r>::run(v[u], sign);
        const int idxd = (j / NS) * NS * r + k;
        cx<T>* base = lds + l * LS;
#pragma unroll
        for (int q = 0; q < r; ++q) base[(idxd + q * NS) * ES] = v[u][q];
      }
    }
    __syncthreads();
    sm_pass<T, N, NL, LF, P + 1, NS * r>(lds, tw, sign, tid);
  }
}

// Unnormalised transform of NL lines in LDS (callers synchronise before;
// the last pass ends with a barrier).  sign -1 forward, +1 inverse.
template <typename T, int N, int NL, bool LF>
__device__ __forceinline__ void sm_fft(cx<T>* lds, const cx<T>* tw, T sign, int tid) {
  sm_pass<T, N, NL, LF, 0, 1>(lds, tw, sign, tid);
}

// x pass of a full-complex field (the runtime-planned xpass_kernel with the
// row length N and NL rows per workgroup fixed): inverse x-FFT, local map of
// the scheme, forward x-FFT, per-workgroup fp64 partial sums.
template <typename T, int N>
__global__ __launch_bounds__(kSmNT) void xpass_sm_kernel(XArgs a) {
  constexpr int NL = sm_lines<T, N>();
  const int solve = blockIdx.z;
  const int comp = blockIdx.y;
  SolveCtl* ctl = a.ctl + solve;
  if (!a.ignore_done && ctl->done) return;
  extern __shared__ unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const int tid = threadIdx.x;
  const long long line0 = (long long)blockIdx.x * NL;
  const int nl = (int)min((long long)NL, (long long)a.nlines - line0);
  const int cnt = nl * N;
  const long long fbase = ((long long)solve * a.d + comp) * a.M;
  const long long base = line0 * N;
  cx<T>* X = reinterpret_cast<cx<T>*>(a.X) + fbase;
  const cx<T>* tw = reinterpret_cast<const cx<T>*>(a.tw);
  // rows past the field's last one (tail workgroup) transform zeros
  for (int i = tid; i < NL * N; i += kSmNT) lds[i] = i < cnt ? X[base + i] : mk<T>(0, 0);
  __syncthreads();
  sm_fft<T, N, NL, false>(lds, tw, (T)1, tid);
  LocalMap<T> lm;
  lm.load(a, solve, comp, fbase);
  Acc acc;
  for (int i = tid; i < cnt; i += kSmNT) lds[i] = lm.apply(lds[i], base + i, acc);
  __syncthreads();
  sm_fft<T, N, NL, false>(lds, tw, (T)-1, tid);
  for (int i = tid; i < cnt; i += kSmNT) X[base + i] = lds[i];
  // deterministic workgroup reduction (wave64 shuffles, then across waves)
  double v[5] = {acc.Jr, acc.Ji, acc.e2, acc.d2, acc.eJ};
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    double s = v[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    v[k] = s;
  }
  __syncthreads();   // every thread has stored its outputs: the LDS is free
  double* red = reinterpret_cast<double*>(smem_raw);   // [5][kSmNT/64]
  const int lane = tid & 63, wave = tid >> 6;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 5; ++k) red[k * (kSmNT / 64) + wave] = v[k];
  }
  __syncthreads();
  if (tid < 5) {
    double s = 0;
    for (int w = 0; w < kSmNT / 64; ++w) s += red[tid * (kSmNT / 64) + w];
    a.part[(((long long)solve * a.d + comp) * 5 + tid) * gridDim.x + blockIdx.x] = s;
  }
}

// Gamma pass of a 2D full-complex field (the runtime-planned
// line_pass_kernel in mode 0 with the column length N and the tile width C
// fixed): forward y-FFT of both components of C adjacent columns, Gamma_1 of
// eq. J11 (J44-J45 in H'') with the scheme's k = 0 source, inverse y-FFT.
// LDS layout [k][line], line = comp*C + l.  Workgroup (0, 0) of each solve
// also reduces the x pass's partial sums and applies the stop rules.
template <typename T, int N>
__global__ __launch_bounds__(kSmNT) void gamma_sm_kernel(GArgs a) {
  constexpr int C = sm_cols<T, N>();
  constexpr int W = 2 * C;
  const int solve = blockIdx.z;
  SolveCtl* ctl = a.ctl + solve;
  if (!a.ignore_done && ctl->done) return;
  extern __shared__ unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const int tid = threadIdx.x;
  if (a.fin && blockIdx.x == 0) finalize_solve(a.f, solve, tid, kSmNT);
  const int x0 = blockIdx.x * C;
  const int nlc = min(C, a.n[0] - x0);
  const long long M = a.M;
  cx<T>* X = reinterpret_cast<cx<T>*>(a.X) + (long long)solve * 2 * M + x0;
  const cx<T>* tw = reinterpret_cast<const cx<T>*>(a.tw);
  const long long stride = a.stride;
  for (int i = tid; i < N * W; i += kSmNT) {
    const int k = i / W;
    const int r = i - k * W;
    const int c = r / C;
    const int l = r - c * C;
    lds[i] = l < nlc ? X[c * M + (long long)k * stride + l] : mk<T>(0, 0);
  }
  __syncthreads();
  sm_fft<T, N, W, true>(lds, tw, (T)-1, tid);
  const SolveCoef& cf = a.coef[solve];
  const T ga = (T)cf.ga, gb = (T)cf.gb, keep = (T)cf.kz_keep;
  for (int i = tid; i < N * C; i += kSmNT) {
    const int k = i / C;
    const int l = i - k * C;
    if (l >= nlc) continue;
    const int m[3] = {x0 + l, k, 0};
    T tv[2][2];
    symbol_entries<T, 2>(a, m, tv);
    cx<T> w[2] = {lds[k * W + l], lds[k * W + C + l]};
    gamma_mode<T, 2>(a, cf, ga, gb, keep, m, tv, w);
    lds[k * W + l] = w[0];
    lds[k * W + C + l] = w[1];
  }
  __syncthreads();
  sm_fft<T, N, W, true>(lds, tw, (T)1, tid);
  for (int i = tid; i < N * W; i += kSmNT) {
    const int k = i / W;
    const int r = i - k * W;
    const int c = r / C;
    const int l = r - c * C;
    if (l < nlc) X[c * M + (long long)k * stride + l] = lds[i];
  }
}

}  // namespace scfft
