// Compile-time mixed-radix passes for 2/3/5-smooth line lengths (gfx950).
//
// Each line is transformed by LW lanes of one wave (all 64, or 32 / 16 for
// short lines, several lines to a wave) through its own LDS slot, so the
// Stockham passes synchronise only the wave (an in-order LDS queue plus a
// compiler fence), never the workgroup; the line length, the radix
// sequence and the slot layout are compile-time constants, so every pass is
// unrolled and its index arithmetic folds into multiplications by constants.
// Workgroup barriers remain only where waves exchange data: the staging of
// the strided Gamma tile (coalesced row segments) and the Gamma step, which
// couples the components of one mode.  One instantiation per supported length
// (SCFFT_SMOOTH_SWITCH); other smooth lengths keep the runtime-planned
// passes.
//
// Stockham pass p with radix r and stride NS (product of the earlier radices)
// maps butterfly j (0 <= j < N/r) from inputs j + q N/r to outputs
// (j div NS) NS r + (j mod NS) + q NS after twiddles exp(-+2 pi i (j mod NS)
// q / (NS r)); unnormalised, forward exp(-2 pi i jk/N).
#pragma once

#include "kernels_real.hpp"

namespace scfft {

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

// Lane slots a line of n points occupies over its passes when each pass's
// butterflies are dealt to lw lanes (a pass of b butterflies costs
// ceil(b / lw) lw slots).
constexpr int sm_slots(int n, int lw) {
  int s = 0;
  for (int p = 0; sm_radix(n, p) > 0; ++p) {
    const int b = n / sm_radix(n, p);
    s += (b + lw - 1) / lw * lw;
  }
  return s;
}

// Lanes per line: 64, or 32 / 16 (several lines to a wave) while that saves
// at least 15 % of the lane slots (a 64-lane 240-point line fills 30 lanes
// in its radix-8 pass; 32-lane lines cut its slots from 384 to 320).
constexpr int sm_lanes(int n) {
  int lw = 64;
  if (sm_slots(n, 32) * 100 <= sm_slots(n, 64) * 85) {
    lw = 32;
    if (sm_slots(n, 16) * 100 <= sm_slots(n, 32) * 85) lw = 16;
  }
  return lw;
}

// Orders this wave's LDS accesses: every lane's earlier reads and writes
// are complete (and visible to the wave) before any later one.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Per-length layout: a line's slot holds N points plus a pad that puts
// consecutive slots one bank apart (slot stride = 1 mod 64 banks per point).
template <typename T, int N>
struct SmShape {
  static constexpr int DW = (int)sizeof(cx<T>) / 4;   // dwords per point
  static constexpr int Q = 64 / DW;                  // points per bank sweep
  static constexpr int LSP = (N + Q - 2) / Q * Q + 1;
  static constexpr int R0 = sm_radix(N, 0);          // radix of the first pass
  static constexpr int LW = sm_lanes(N);              // lanes per line
  static constexpr int LPW = 64 / LW;                // lines per wave
  static constexpr int B0 = (N / R0 + LW - 1) / LW;  // first-pass butterflies per lane
  // x pass: waves per workgroup (measured on the 16-grid batch: two beat
  // four; one for short lines, so that small grids keep their workgroup
  // count), XL rows
  static constexpr int XW = LPW > 1 ? 1 : 2;
  static constexpr int XL = XW * LPW;
  static constexpr int XLDS = XL * LSP * (int)sizeof(cx<T>) + 5 * XW * 8;
};

// Strided passes: tiles of C adjacent columns, one line (LW lanes) per
// column and component (D components: 2 / 3 the Gamma pass of a 2D / 3D
// grid, 1 a plain 3D y pass).  2D Gamma, measured on the 16-grid batch:
// 8 fp32 columns (64-byte row pieces) beat 4 by 8 %; fp64 keeps 2.  The y
// pass takes 64-byte pieces in both precisions; the 3D Gamma pass halves
// the 2D widths to stay within 16 waves.  In 3D, lines of fewer than 64
// lanes widen the tile by the lines per wave; 2D grids of short lines have
// few columns, and keep their tile count.
template <typename T, int N, int D>
struct SmTile {
  static constexpr bool F = sizeof(T) == 4;
  static constexpr int LW = SmShape<T, N>::LW;
  static constexpr int C = (D == 1 ? (F ? 8 : 4) : D == 2 ? (F ? 8 : 2) : (F ? 4 : 2)) *
                           (D == 2 ? 1 : SmShape<T, N>::LPW);
  static constexpr int GW = D * C;                   // lines per workgroup
  static constexpr int NT = GW * LW;                 // threads
  static constexpr int LDS = GW * SmShape<T, N>::LSP * (int)sizeof(cx<T>);
  static_assert(NT <= 1024, "at most 1024 threads per workgroup");
};

// One radix-r pass of a line held by LW lanes of a wave (slot: N points at
// slot[0..N); lane: 0..LW-1).  P = 0 takes its inputs from the registers v0
// (point j + q N/R0 of butterfly j = lane + LW u at v0[u][q]); every pass
// writes its outputs to the slot.
template <typename T, int N, int P, int NS>
__device__ __forceinline__ void sm_pass(const cx<T> (&v0)[SmShape<T, N>::B0][SmShape<T, N>::R0],
                                        cx<T>* __restrict__ slot, const cx<T>* __restrict__ tw,
                                        T sign, int lane) {
  if constexpr (NS < N) {
    constexpr int r = sm_radix(N, P);
    static_assert(r > 0 && N % (NS * r) == 0, "radix sequence must factor N");
    constexpr int LW = SmShape<T, N>::LW;
    constexpr int NBL = N / r;                  // butterflies
    constexpr int BPL = (NBL + LW - 1) / LW;    // per lane
    constexpr int STEP = N / (NS * r);          // twiddle table stride
    cx<T> v[BPL][r];
    if constexpr (P == 0) {
#pragma unroll
      for (int u = 0; u < BPL; ++u)
#pragma unroll
        for (int q = 0; q < r; ++q) v[u][q] = v0[u][q];
    } else {
#pragma unroll
      for (int u = 0; u < BPL; ++u) {
        const int j = lane + LW * u;
        if (NBL % LW == 0 || j < NBL) {
#pragma unroll
          for (int q = 0; q < r; ++q) v[u][q] = slot[j + q * NBL];
        }
      }
    }
    wave_sync();   // the pass's reads are done before its in-place writes
#pragma unroll
    for (int u = 0; u < BPL; ++u) {
      const int j = lane + LW * u;
      if (NBL % LW == 0 || j < NBL) {
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
#pragma unroll
        for (int q = 0; q < r; ++q) slot[idxd + q * NS] = v[u][q];
      }
    }
    wave_sync();
    sm_pass<T, N, P + 1, NS * r>(v0, slot, tw, sign, lane);
  }
}

// Unnormalised transform of one line held by LW lanes: input in registers in
// the first pass's layout, output in the slot in natural order (sign -1
// forward, +1 inverse).
template <typename T, int N>
__device__ __forceinline__ void sm_fft(const cx<T> (&v0)[SmShape<T, N>::B0][SmShape<T, N>::R0],
                                       cx<T>* slot, const cx<T>* tw, T sign, int lane) {
  sm_pass<T, N, 0, 1>(v0, slot, tw, sign, lane);
}

// x pass of a full-complex field: one row per LW lanes, XL rows per
// workgroup (rows past the field's last transform zeros and are not
// stored): inverse
// x-FFT, local map of the scheme (MK fixes it at compile time), forward
// x-FFT, fp64 partial sums.
template <typename T, int N, int MK>
__global__ __launch_bounds__((64 * SmShape<T, N>::XW)) void xpass_sm_kernel(XArgs a) {
  using SH = SmShape<T, N>;
  constexpr int R0 = SH::R0, B0 = SH::B0, NB0 = N / R0, LW = SH::LW;
  const int solve = blockIdx.z;
  const int comp = blockIdx.y;
  if (!a.ignore_done && a.ctl[solve].done) return;
  extern __shared__ unsigned char smem_raw[];
  const int tid = threadIdx.x, lane = tid % LW, w = tid / LW;
  cx<T>* slot = reinterpret_cast<cx<T>*>(smem_raw) + w * SH::LSP;
  double* red = reinterpret_cast<double*>(smem_raw + SH::XL * SH::LSP * sizeof(cx<T>));
  const long long line = (long long)blockIdx.x * SH::XL + w;
  const bool valid = line < a.nlines;
  const long long fbase = ((long long)solve * a.d + comp) * a.M;
  const long long base = line * N;
  cx<T>* X = reinterpret_cast<cx<T>*>(a.X) + fbase;
  const cx<T>* tw = reinterpret_cast<const cx<T>*>(a.tw);
  cx<T> v0[B0][R0];
#pragma unroll
  for (int u = 0; u < B0; ++u) {
    const int j = lane + LW * u;
#pragma unroll
    for (int q = 0; q < R0; ++q)
      v0[u][q] = (valid && (NB0 % LW == 0 || j < NB0)) ? X[base + j + q * NB0] : mk<T>(0, 0);
  }
  LocalMap<T, MK> lm;
  lm.load(a, solve, comp, fbase);
  // the phase map and E_prev do not depend on the FFT: load them first when
  // the registers allow (at most 16 fp32 / 8 fp64 points per lane)
  constexpr bool PF = (MK == MAP_LIN || MK == MAP_ACC_EM || MK == MAP_ACC_MS) &&
                      B0 * R0 * (int)sizeof(cx<T>) <= 128;
  bool ph[PF ? B0 : 1][PF ? R0 : 1];
  cx<T> epo[PF ? B0 : 1][PF ? R0 : 1];
  if (PF && valid) {
#pragma unroll
    for (int u = 0; u < B0; ++u) {
      const int j = lane + LW * u;
      if (NB0 % LW == 0 || j < NB0) {
#pragma unroll
        for (int q = 0; q < R0; ++q) {
          const long long g = base + j + q * NB0;
          ph[PF ? u : 0][PF ? q : 0] = lm.phase[g] != 0;
          epo[PF ? u : 0][PF ? q : 0] = lm.Ep[g];
        }
      }
    }
  }
  sm_fft<T, N>(v0, slot, tw, (T)1, lane);
  Acc acc;
#pragma unroll
  for (int u = 0; u < B0; ++u) {
    const int j = lane + LW * u;
    if (valid && (NB0 % LW == 0 || j < NB0)) {
#pragma unroll
      for (int q = 0; q < R0; ++q) {
        const long long g = base + j + q * NB0;
        v0[u][q] = PF ? lm.apply_pf(slot[j + q * NB0], g, ph[PF ? u : 0][PF ? q : 0],
                                    epo[PF ? u : 0][PF ? q : 0], acc)
                      : lm.apply(slot[j + q * NB0], g, acc);
        acc_settle<true>(acc);
      }
    }
  }
  sm_fft<T, N>(v0, slot, tw, (T)-1, lane);
  if (valid) {
#pragma unroll
    for (int t = 0; t < (N + LW - 1) / LW; ++t) {
      const int i = lane + LW * t;
      if (N % LW == 0 || i < N) X[base + i] = slot[i];
    }
  }
  block_reduce5<64 * SH::XW>(acc, red,
                             a.part + ((long long)solve * a.d + comp) * 5 * gridDim.x + blockIdx.x,
                             gridDim.x, tid);
}

// x pass of a real field (real-field mode): each line is the pair of real
// rows (2p, 2p + 1) of one component, transformed as w = a + i b, XL pairs
// per workgroup.  The half spectra A(k), B(k) (k = 0..N/2, no packed
// column) give W(k) = A(k) + i B(k), with A(N - k) = conj A(k) above N/2;
// inverse FFT, the real local map on a and b, forward FFT, and the rows'
// half spectra back from A = (W(k) + conj W(N-k)) / 2,
// B = (W(k) - conj W(N-k)) / 2i; fp64 partial sums.
template <typename T, int N, int MK>
__global__ __launch_bounds__((64 * SmShape<T, N>::XW)) void xpass_sm_r2c_kernel(XArgs a) {
  using SH = SmShape<T, N>;
  constexpr int R0 = SH::R0, B0 = SH::B0, NB0 = N / R0, LW = SH::LW;
  static_assert(N % 2 == 0, "real rows of even length");
  const int solve = blockIdx.z;
  const int comp = blockIdx.y;
  if (!a.ignore_done && a.ctl[solve].done) return;
  extern __shared__ unsigned char smem_raw[];
  const int tid = threadIdx.x, lane = tid % LW, w = tid / LW;
  cx<T>* slot = reinterpret_cast<cx<T>*>(smem_raw) + w * SH::LSP;
  double* red = reinterpret_cast<double*>(smem_raw + SH::XL * SH::LSP * sizeof(cx<T>));
  const long long pr = (long long)blockIdx.x * SH::XL + w;
  const bool valid = pr < a.nlines / 2;
  const long long rowA = 2 * pr, rowB = 2 * pr + 1;
  const long long cbase = (long long)solve * a.d + comp;
  cx<T>* XA = reinterpret_cast<cx<T>*>(a.X) + cbase * a.Mh + rowA * a.hp;
  cx<T>* XB = XA + a.hp;
  const cx<T>* tw = reinterpret_cast<const cx<T>*>(a.tw);
  cx<T> v0[B0][R0];
#pragma unroll
  for (int u = 0; u < B0; ++u) {
    const int j = lane + LW * u;
#pragma unroll
    for (int q = 0; q < R0; ++q) {
      const int k = j + q * NB0;
      cx<T> av = mk<T>(0, 0), bv = mk<T>(0, 0);
      if (valid && (NB0 % LW == 0 || j < NB0)) {
        if (k <= N / 2) {
          av = XA[k];
          bv = XB[k];
        } else {
          av = conj(XA[N - k]);
          bv = conj(XB[N - k]);
        }
      }
      v0[u][q] = mk<T>(av.x - bv.y, av.y + bv.x);   // a + i b
    }
  }
  LocalMapR<T, MK> lm;
  lm.load(a, solve, comp, cbase * a.M);
  const auto wa = lm.row(rowA * N);
  const auto wb = lm.row(rowB * N);
  // the phase maps and E_prev do not depend on the FFT: load them first
  // when the registers allow (at most 16 fp32 / 8 fp64 points per lane)
  constexpr bool PF = (MK == MAP_LIN || MK == MAP_ACC_EM || MK == MAP_ACC_MS) &&
                      B0 * R0 * (int)sizeof(cx<T>) <= 128;
  constexpr int PB = PF ? B0 : 1, PR = PF ? R0 : 1;
  // the H'' slots of phase-1 voxels too, for up to 8 fp32 points per lane
  constexpr bool PSL = PF && sizeof(T) == 4 && B0 * R0 <= 8;
  constexpr bool PS = PSL && (MK == MAP_ACC_EM || MK == MAP_ACC_MS);
  constexpr bool PT = PSL && MK == MAP_ACC_EM;
  bool pha[PB][PR], phb[PB][PR];
  T epa[PB][PR], epb[PB][PR];
  T sa[PB][PR], sb[PB][PR], ta[PB][PR], tb[PB][PR];
  if (PF && valid) {
#pragma unroll
    for (int u = 0; u < B0; ++u) {
      const int j = lane + LW * u;
      if (NB0 % LW == 0 || j < NB0) {
#pragma unroll
        for (int q = 0; q < R0; ++q) {
          const unsigned int k = (unsigned int)(j + q * NB0);
          const int pu = PF ? u : 0, pq = PF ? q : 0;
          pha[pu][pq] = wa.ph[k] != 0;
          phb[pu][pq] = wb.ph[k] != 0;
          epa[pu][pq] = wa.Ep[k];
          epb[pu][pq] = wb.Ep[k];
        }
#pragma unroll
        for (int q = 0; q < R0; ++q) {
          const unsigned int k = (unsigned int)(j + q * NB0);
          const int pu = PF ? u : 0, pq = PF ? q : 0;
          sa[pu][pq] = (PS && pha[pu][pq]) ? wa.S[k] : (T)0;
          sb[pu][pq] = (PS && phb[pu][pq]) ? wb.S[k] : (T)0;
          ta[pu][pq] = (PT && pha[pu][pq]) ? wa.Tt[k] : (T)0;
          tb[pu][pq] = (PT && phb[pu][pq]) ? wb.Tt[k] : (T)0;
        }
      }
    }
  }
  sm_fft<T, N>(v0, slot, tw, (T)1, lane);
  Acc acc;
#pragma unroll
  for (int u = 0; u < B0; ++u) {
    const int j = lane + LW * u;
    if (valid && (NB0 % LW == 0 || j < NB0)) {
#pragma unroll
      for (int q = 0; q < R0; ++q) {
        const unsigned int k = (unsigned int)(j + q * NB0);
        const cx<T> z = slot[k];
        const int pu = PF ? u : 0, pq = PF ? q : 0;
        const T oa = PF ? lm.template apply_pf<PSL>(z.x, pha[pu][pq], epa[pu][pq], sa[pu][pq],
                                                    ta[pu][pq], wa, k, acc)
                        : lm.apply(z.x, wa, k, acc);
        const T ob = PF ? lm.template apply_pf<PSL>(z.y, phb[pu][pq], epb[pu][pq], sb[pu][pq],
                                                    tb[pu][pq], wb, k, acc)
                        : lm.apply(z.y, wb, k, acc);
        v0[u][q] = mk<T>(oa, ob);
        acc_settle<false>(acc);
      }
    }
  }
  sm_fft<T, N>(v0, slot, tw, (T)-1, lane);
  if (valid) {
#pragma unroll
    for (int t = 0; t < (N / 2 + LW) / LW; ++t) {
      const int k = lane + LW * t;
      if (k <= N / 2) {
        const cx<T> wk = slot[k];
        const cx<T> wn = conj(slot[k == 0 ? 0 : N - k]);
        const cx<T> sm = wk + wn, df = wk - wn;
        XA[k] = mk<T>((T)0.5 * sm.x, (T)0.5 * sm.y);
        XB[k] = mk<T>((T)0.5 * df.y, (T)-0.5 * df.x);
      }
    }
  }
  block_reduce5<64 * SH::XW>(acc, red, a.part + cbase * 5 * gridDim.x + blockIdx.x, gridDim.x,
                             tid);
}

// Strided pass over the columns of the spectrum (n0 of a full-complex
// field, n0/2 + 1 in real-field mode) along lines of N points on the last
// axis (a.mode 0: forward FFT, Gamma_1 of eq. J11 (J44-J45 in H'') with
// the scheme's k = 0 source, inverse FFT, all D = d components) or along y in
// 3D (mode 1 / 2: forward / inverse FFT of one component, D = 1).  A tile of
// C adjacent columns, one line of LW lanes per column and component: the
// tile is staged through LDS in row pieces, each line is transformed by its
// own lanes, the Gamma
// step couples the components of every mode, and the tile is stored back.
// Workgroup (0, 0) of each solve's Gamma pass also reduces the x pass's
// partial sums and applies the stop rules.
template <typename T, int N, int D>
__global__ __launch_bounds__((SmTile<T, N, D>::NT)) void line_sm_kernel(GArgs a) {
  using SH = SmShape<T, N>;
  using TS = SmTile<T, N, D>;
  constexpr int R0 = SH::R0, B0 = SH::B0, NB0 = N / R0, LSP = SH::LSP, LW = SH::LW;
  constexpr int C = TS::C, GW = TS::GW, NT = TS::NT;
  const bool gam = (a.mode == 0);
  const int d = a.d;
  const int solve = gam ? blockIdx.z : blockIdx.z / d;
  const int comp0 = gam ? 0 : blockIdx.z % d;
  if (!a.ignore_done && a.ctl[solve].done) return;
  extern __shared__ unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const int tid = threadIdx.x, lane = tid % LW, w = tid / LW;
  if (a.fin && blockIdx.x == 0 && blockIdx.y == 0 && comp0 == 0)
    finalize_solve(a.f, solve, tid, NT);
  // XCD-aware tile order: the hardware deals workgroups round-robin over
  // the 8 XCDs, so consecutive tiles (sharing cache lines at their edges)
  // are given to workgroups that run on the same XCD and L2 (measured: the
  // fp32 3D Gamma pass 24 % faster at 240^3 and 320^3)
  const int nbx = gridDim.x, nb = nbx * gridDim.y;
  const int b = blockIdx.y * nbx + blockIdx.x;
  const int full = nb - nb % 8;
  const int t = b < full ? (b % 8) * (full / 8) + b / 8 : b;
  const int bx = t % nbx, by = t / nbx;
  const int x0 = bx * C;
  const int nlc = min(C, a.n[0] - x0);
  const long long M = a.M;
  // 2D Gamma: x0; 3D Gamma: x0 + y rp; 3D y pass: x0 + z rp n1
  const long long off = x0 + (long long)by * a.rp * (gam ? 1 : a.n[1]);
  cx<T>* X = reinterpret_cast<cx<T>*>(a.X) + ((long long)solve * d + comp0) * M + off;
  const cx<T>* tw = reinterpret_cast<const cx<T>*>(a.tw);
  const long long stride = a.stride;
  // line w = comp * C + column; its slot at lds + w * LSP
#pragma unroll 4
  for (int i = tid; i < N * GW; i += NT) {
    const int k = i / GW;
    const int r = i - k * GW;
    const int c = r / C;
    const int l = r - c * C;
    lds[r * LSP + k] = l < nlc ? X[c * M + (long long)k * stride + l] : mk<T>(0, 0);
  }
  __syncthreads();
  cx<T>* slot = lds + w * LSP;
  cx<T> v0[B0][R0];
  if (a.mode != 2) {
#pragma unroll
    for (int u = 0; u < B0; ++u) {
      const int j = lane + LW * u;
      if (NB0 % LW == 0 || j < NB0) {
#pragma unroll
        for (int q = 0; q < R0; ++q) v0[u][q] = slot[j + q * NB0];
      }
    }
    sm_fft<T, N>(v0, slot, tw, (T)-1, lane);
  }
  if constexpr (D > 1) {
    __syncthreads();
    const SolveCoef& cf = a.coef[solve];
    const T ga = (T)cf.ga, gb = (T)cf.gb, keep = (T)cf.kz_keep;
    for (int i = tid; i < N * C; i += NT) {
      const int k = i / C;
      const int l = i - k * C;
      if (l >= nlc) continue;
      const int m[3] = {x0 + l, D == 2 ? k : by, D == 2 ? 0 : k};
      T tv[D][2];
      symbol_entries<T, D>(a, m, tv);
      cx<T> wv[D];
#pragma unroll
      for (int c = 0; c < D; ++c) wv[c] = lds[(c * C + l) * LSP + k];
      gamma_mode<T, D>(a, cf, ga, gb, keep, m, tv, wv);
#pragma unroll
      for (int c = 0; c < D; ++c) lds[(c * C + l) * LSP + k] = wv[c];
    }
    __syncthreads();
  }
  if (a.mode != 1) {
#pragma unroll
    for (int u = 0; u < B0; ++u) {
      const int j = lane + LW * u;
      if (NB0 % LW == 0 || j < NB0) {
#pragma unroll
        for (int q = 0; q < R0; ++q) v0[u][q] = slot[j + q * NB0];
      }
    }
    sm_fft<T, N>(v0, slot, tw, (T)1, lane);
  }
  __syncthreads();
#pragma unroll 4
  for (int i = tid; i < N * GW; i += NT) {
    const int k = i / GW;
    const int r = i - k * GW;
    const int c = r / C;
    const int l = r - c * C;
    if (l < nlc) X[c * M + (long long)k * stride + l] = lds[r * LSP + k];
  }
}

}  // namespace scfft
