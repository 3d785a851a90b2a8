// Host driver and C ABI of libscfft (see include/scfft.h).
//
// The host side only validates arguments, computes the scheme scalars in fp64
// (slit map t of eq. J23, p of eq. J24, the expansion variables of eqs. J1,
// J2, J4, J42a), owns cached device workspaces, and enqueues the kernels of
// kernels.hpp; every per-voxel and per-mode operation runs on the GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "kernels_lanczos.hpp"
#include "launch.hpp"
#include "scfft.h"

using cd = std::complex<double>;

namespace scfft {
namespace {

constexpr int kNT = 1024;
// elements a workgroup transforms at once (64 KiB of LDS in both precisions)
constexpr int kElemsF32 = 8192;
constexpr int kElemsF64 = 4096;

#define SCFFT_HIP(call)                                                     \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess) {                                                 \
      if (std::getenv("SCFFT_LOG"))                                         \
        std::fprintf(stderr, "scfft: %s failed: %s (%s:%d)\n", #call,       \
                     hipGetErrorString(e_), __FILE__, __LINE__);            \
      return e_ == hipErrorOutOfMemory ? SCFFT_ERR_OOM : SCFFT_ERR_DEVICE;  \
    }                                                                       \
  } while (0)

bool smooth235(int n) {
  if (n < 2) return false;
  for (int p : {2, 3, 5})
    while (n % p == 0) n /= p;
  return n == 1;
}

FftDesc make_desc(int n) {
  FftDesc fd{};
  fd.n = n;
  int m = n;
  for (int r : {8, 4, 2, 3, 5}) {
    while (m % r == 0) {
      fd.radix[fd.npass++] = r;
      m /= r;
    }
  }

  return fd;
}

int pow2_floor(int v) {
  int p = 1;
  while (p * 2 <= v) p *= 2;
  return p;
}


// MI355X Infinity Cache (last-level cache in front of HBM)
constexpr size_t kInfinityCacheBytes = (size_t)256 << 20;

bool is_p2(int n) { return n >= 16 && n <= 4096 && (n & (n - 1)) == 0; }


// 2D real mode: pack kx = 0 and kx = n0/2 into one column when that lowers
// the number of Gamma-pass workgroups the busiest CU runs (the packed tile
// does a little more work, so packing only pays where it removes a tile
// from some CU).
bool pack_pays(int n0, int c, int nsolve, int dev) {
  if (const char* e = std::getenv("SCFFT_PACK")) return std::atoi(e) != 0;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    return false;
  const long long tu = (long long)nsolve * ((n0 / 2 + 1 + c - 1) / c);
  const long long tp = (long long)nsolve * ((n0 / 2 + c - 1) / c);
  return (tu + cus - 1) / cus > (tp + cus - 1) / cus;
}

// ------------------------------------------------------------ plan knobs
// Speed choices of a plan.  Every value gives the same iterates up to
// rounding (each is parity-tested); 0 / -1 means "the measured rule" below.
struct Knobs {
  int xr = 0;      // x pass register radix: 4 or 8
  int gr = 0;      // Gamma pass register radix: 2D 4 or 8 (fp64 2048-point lines also 16); 3D 8
  int gC = 0;      // Gamma pass tile width: 1, 2, 4, 8 (capped by the LDS budget)
  int yC = 0;      // 3D y pass tile width: 1, 2, 4, 8
  int pack = -1;   // 2D real mode: kx = 0 and n0/2 share column 0
  int nt = -1;     // real mode: the x pass streams its own arrays nontemporally
  int pitch = -1;  // real mode: rows of X padded to 128-byte lines
  bool operator==(const Knobs& o) const {
    return xr == o.xr && gr == o.gr && gC == o.gC && yC == o.yC && pack == o.pack && nt == o.nt &&
           pitch == o.pitch;
  }
};

// Environment overrides force a knob (tests force each candidate this way).
int env_int(const char* name, int dflt) {
  const char* e = std::getenv(name);
  return e ? std::atoi(e) : dflt;
}

// Register radix rules (measured on MI355X, fp32 and fp64): radix 4 (twice
// the threads per line, more waves in flight) for the x pass up to n0 = 1024
// (fp64: 2048) and for the 2D Gamma pass up to 1024; radix 8 (fewer LDS
// exchanges) for longer lines and the 3D strided passes; radix 16 (one
// exchange fewer again) for the fp64 Gamma pass of 2048-point lines
// (115 -> 104 us).
int rule_xr(int n, int esz) { return (n <= 1024 || (esz == 16 && n <= 2048)) ? 4 : 8; }
int rule_gr(int n, int esz, int d) {
  if (d != 2) return 8;
  if (esz == 16 && n == 2048 && env_int("SCFFT_R16", 1) != 0) return 16;
  return n <= 1024 ? 4 : 8;
}

struct Plan {
  int HP = 0;        // row pitch of X in elements (real mode: H rounded up to a cache line)
  bool nt = false;   // real-mode x pass streams its own arrays nontemporally
  int dev = 0, d = 2, n[3] = {1, 1, 1}, prec = 0, nsolve = 1, symbol = 0;
  bool st = false;
  long long M = 0;
  size_t esz = 16;
  void* X = nullptr;
  void* Ep = nullptr;
  void* S = nullptr;
  void* T = nullptr;
  double* part = nullptr;
  SolveCtl* ctl = nullptr;
  SolveCoef* coef = nullptr;
  double* hist_r = nullptr;
  double* hist_s = nullptr;
  int hist_cap = 0;
  void* tw[3] = {nullptr, nullptr, nullptr};
  double* sym[3] = {nullptr, nullptr, nullptr};
  FftDesc fd[3];
  int xlines = 0, xL = 1, xblocks = 0;
  int gC = 1, yC = 1;
  bool p2x = false, p2g = false, p2y = false;   // register-resident passes
  bool smx = false, smg = false, smy = false;    // compile-time mixed-radix passes
  Knobs kn;                                      // resolved speed choices
  bool tuned = false;                            // kn came from the autotuner
  int mk = MAP_LIN;                              // local map of the current solves
  bool no_alloc = false;                         // workspace carved from the fixed array
  SolveCtl* ctl_host = nullptr;                  // pinned: the loop's stop-flag reads
  bool real = false;                             // real-field mode (half spectra)
  bool packed = false;                           // 2D real mode: kx = 0 and n0/2 share column 0
  int H = 0;                                     // stored x-spectrum length
  long long Mh = 0;                              // stored elements per component of X
  size_t xbytes = 0, rbytes = 0;                 // X; each real-space array (E_prev, S, T)
};

int map_kind(int kind, bool density) {
  if (kind == K_ACC_EM) return MAP_ACC_EM;
  if (kind == K_ACC_MS) return MAP_ACC_MS;
  return density ? MAP_LIN_DENS : MAP_LIN;
}

using PlanKey = std::tuple<int, int, int, int, int, int, int, bool, int, int, bool>;
std::map<PlanKey, Plan*> g_plans;
std::mutex g_mutex;

void free_plan(Plan* p) {
  if (!p) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(p->dev);
  void* ptrs[] = {p->X, p->Ep, p->S, p->T, p->part, p->ctl, p->coef, p->hist_r, p->hist_s,
                  p->tw[0], p->tw[1], p->tw[2], p->sym[0], p->sym[1], p->sym[2]};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  if (p->ctl_host) (void)hipHostFree(p->ctl_host);
  (void)hipSetDevice(cur);
  delete p;
}

int elems_for(int prec) { return prec == SCFFT_FP32 ? kElemsF32 : kElemsF64; }

// Size limits of the LDS-staged passes.
scfft_status check_dims(int d, const int* n, int prec) {
  if (d != 2 && d != 3) return SCFFT_ERR_INVALID_ARG;
  for (int i = 0; i < d; ++i)
    if (!smooth235(n[i]) || n[i] > 4096) return SCFFT_ERR_INVALID_ARG;
  const int el = elems_for(prec);
  if (n[0] > el) return SCFFT_ERR_INVALID_ARG;
  if (n[d - 1] * d > el) return SCFFT_ERR_INVALID_ARG;
  if (d == 3 && n[1] > el) return SCFFT_ERR_INVALID_ARG;
  return SCFFT_OK;
}

scfft_status ensure_hist(Plan* p, int need) {
  if (need <= p->hist_cap) return SCFFT_OK;
  if (need > (1 << 27)) return SCFFT_ERR_OOM;
  // room for at least 1024 iterates, in powers of two: solves of other
  // lengths then reuse the buffers, and with them the captured graphs
  int cap = 1024;
  while (cap < need) cap *= 2;
  if (p->hist_r) (void)hipFree(p->hist_r);
  if (p->hist_s) (void)hipFree(p->hist_s);
  p->hist_r = nullptr;
  p->hist_s = nullptr;
  p->hist_cap = 0;
  SCFFT_HIP(hipMalloc(&p->hist_r, sizeof(double) * (size_t)cap * p->nsolve));
  SCFFT_HIP(hipMalloc(&p->hist_s, 2 * sizeof(double) * (size_t)cap * p->nsolve));
  p->hist_cap = cap;
  return SCFFT_OK;
}

// Every execution-path choice and buffer size of a plan (host only, no
// device work besides reading the compute-unit count).  `want` holds the
// tuner's choices (unset fields follow the rules); environment overrides
// win over both.
void plan_shape(Plan* p, int dev, int d, const int* n, int prec, int nsolve, bool st, int symbol,
                bool real, const Knobs& want = Knobs()) {
  const int n2 = d == 3 ? n[2] : 1;
  p->dev = dev;
  p->d = d;
  p->n[0] = n[0];
  p->n[1] = n[1];
  p->n[2] = n2;
  p->prec = prec;
  p->nsolve = nsolve;
  p->st = st;
  p->symbol = symbol;
  p->M = (long long)n[0] * n[1] * n2;
  p->esz = prec == SCFFT_FP32 ? 8 : 16;
  p->real = real;
  const int esz = (int)p->esz;
  const int el = elems_for(prec);
  const int nlast = n[d - 1];
  p->xlines = (int)(p->M / n[0]);
  p->p2x = is_p2(n[0]) && !std::getenv("SCFFT_NO_P2");
  p->p2g = is_p2(nlast) && !std::getenv("SCFFT_NO_P2") && (d == 2 || nlast <= 1024);
  p->H = real ? n[0] / 2 + 1 : n[0];
  p->p2y = d == 3 && is_p2(n[1]) && !std::getenv("SCFFT_NO_P2");
  const bool sm_on = !std::getenv("SCFFT_NO_SMOOTH");
  p->smx = sm_on && !p->p2x && smooth_lines(n[0], esz) > 0;
  p->smg = sm_on && !p->p2g && smooth_cols(nlast, esz, d) > 0;
  p->smy = sm_on && d == 3 && !p->p2y && smooth_cols(n[1], esz, 1) > 0;
  Knobs& k = p->kn;
  k = Knobs();
  // x pass radix
  if (p->p2x) {
    k.xr = env_int("SCFFT_XR", want.xr ? want.xr : rule_xr(n[0], esz));
    if (k.xr != 4 && k.xr != 8) k.xr = rule_xr(n[0], esz);
    if (n[0] < k.xr) k.xr = 4;
    p->xL = xpass_lines(n[0], esz, k.xr);
  } else if (p->smx) {
    k.xr = 0;
    p->xL = smooth_lines(n[0], esz);
  } else {
    k.xr = 0;
    p->xL = std::max(1, std::min(el / n[0], p->xlines));
  }
  p->xblocks = real ? (p->xlines / 2 + p->xL - 1) / p->xL : (p->xlines + p->xL - 1) / p->xL;
  // Gamma pass radix and tile width
  if (p->p2g) {
    k.gr = env_int("SCFFT_GR", want.gr ? want.gr : rule_gr(nlast, esz, d));
    const bool r16ok = d == 2 && nlast == 2048 && esz == 16;
    if (d == 3 && k.gr != 4) k.gr = 8;
    if (k.gr == 16 && !r16ok) k.gr = rule_gr(nlast, esz, d) == 16 ? 8 : rule_gr(nlast, esz, d);
    if (k.gr != 4 && k.gr != 8 && k.gr != 16) k.gr = rule_gr(nlast, esz, d);
    if (env_int("SCFFT_R16", 1) == 0 && k.gr == 16) k.gr = 8;
    const int cmax = k.gr == 16 ? line_tile_max(nlast, esz, 2, 16) : line_tile_max(nlast, esz, d, k.gr);
    const int c = env_int("SCFFT_LINE_C", want.gC ? want.gC : cmax);
    k.gC = (c == 1 || c == 2 || c == 4 || c == 8) ? std::min(c, cmax) : cmax;
    if (k.gr == 16) k.gC = cmax;   // one instantiation: the widest tile
  } else if (p->smg) {
    k.gr = 0;
    k.gC = smooth_cols(nlast, esz, d);   // fixed by the instantiation
  } else {
    k.gr = 0;
    const int cmax = std::min(pow2_floor(std::max(1, el / (nlast * d))), n[0]);
    const int c = env_int("SCFFT_LINE_C", want.gC ? want.gC : cmax);
    k.gC = c >= 1 ? std::min(pow2_floor(c), cmax) : cmax;
  }
  p->gC = k.gC;
  // 3D y pass tile width
  if (d == 3 && p->p2y) {
    const int cmax = line_tile_max(n[1], esz, 1, 8);
    const int c = env_int("SCFFT_YC", env_int("SCFFT_LINE_C", want.yC ? want.yC : cmax));
    k.yC = (c == 1 || c == 2 || c == 4 || c == 8) ? std::min(c, cmax) : cmax;
  } else if (d == 3 && p->smy) {
    k.yC = smooth_cols(n[1], esz, 1);   // fixed by the instantiation
  } else if (d == 3) {
    const int cmax = std::min(pow2_floor(std::max(1, el / n[1])), n[0]);
    const int c = env_int("SCFFT_YC", env_int("SCFFT_LINE_C", want.yC ? want.yC : cmax));
    k.yC = c >= 1 ? std::min(pow2_floor(c), cmax) : cmax;
  } else {
    k.yC = 1;
  }
  p->yC = k.yC;
  // 2D real mode: pack kx = 0 and kx = n0/2 into one column (the register
  // x and Gamma passes unpack it); the rule packs when that lowers the number of
  // Gamma-pass workgroups the busiest CU runs, and for the radix-16 pass
  if (real && d == 2 && p->p2g && p->p2x) {
    const int dflt = want.pack >= 0 ? want.pack
                   : (k.gr == 16 || pack_pays(n[0], p->gC, nsolve, dev)) ? 1 : 0;
    k.pack = env_int("SCFFT_PACK", dflt) != 0 ? 1 : 0;
  } else {
    k.pack = 0;
  }
  p->packed = k.pack != 0;
  if (p->packed) p->H = n[0] / 2;
  // real mode: rows of X start on 128-byte cache lines, so that a strided
  // pass's tile of adjacent columns shares lines only with its neighbours in
  // the same row (rule: 3D, where 256^3 gained 178 -> 148 us in the fp32 z
  // pass and 560 -> 440 us in fp64; neutral or slightly slower in 2D)
  {
    const int per_line = 128 / esz;
    k.pitch = real ? (env_int("SCFFT_PITCH", want.pitch >= 0 ? want.pitch : (d == 3 ? 1 : 0)) != 0)
                   : 0;
    p->HP = k.pitch ? (p->H + per_line - 1) / per_line * per_line : p->H;
  }
  p->Mh = (long long)p->HP * n[1] * n2;
  const size_t field = (size_t)nsolve * d * p->M * p->esz;
  // real mode: X holds half spectra, the real-space arrays hold real values
  const size_t xfield = real ? (size_t)nsolve * d * p->Mh * p->esz : field;
  const size_t rfield = real ? field / 2 : field;
  // real mode: the x pass streams the phase map, E_prev and the H'' slots
  // nontemporally (rule: when the half spectrum and E_prev alone exceed the
  // 256 MB Infinity Cache; measured: 256^3 fp32 and fp64 gain, 2048^2 fp32 and
  // fp64 lose, the slots being touched only at phase-1 voxels)
  {
    const size_t foot = xfield + rfield;
    k.nt = (real && !p->smx)
               ? (env_int("SCFFT_NT", want.nt >= 0 ? want.nt : (foot > kInfinityCacheBytes)) != 0)
               : 0;
    p->nt = k.nt != 0;
  }
  p->xbytes = xfield;
  p->rbytes = rfield;
  for (int a = 0; a < d; ++a) p->fd[a] = make_desc(n[a]);
}

// Twiddle and symbol tables of every axis (into the plan's buffers).
scfft_status plan_tables(Plan* p, hipStream_t stream) {
  for (int a = 0; a < p->d; ++a) {
    const int n = p->n[a];
    const int blocks = (n + 255) / 256;
    if (p->prec == SCFFT_FP32)
      hipLaunchKernelGGL(twiddle_kernel<float>, dim3(blocks), dim3(256), 0, stream,
                         reinterpret_cast<cx<float>*>(p->tw[a]), n);
    else
      hipLaunchKernelGGL(twiddle_kernel<double>, dim3(blocks), dim3(256), 0, stream,
                         reinterpret_cast<cx<double>*>(p->tw[a]), n);
    hipLaunchKernelGGL(symbol_table_kernel, dim3(blocks), dim3(256), 0, stream, p->sym[a], n,
                       p->symbol);
  }
  SCFFT_HIP(hipGetLastError());
  return SCFFT_OK;
}

// Allocates the buffers of a shaped plan and fills its tables; the partial
// sums are sized for at least part_blocks x-pass workgroups per component.
scfft_status plan_alloc(Plan* p, hipStream_t stream, int part_blocks = 0) {
  const int d = p->d, nsolve = p->nsolve;
  auto fail = [&](hipError_t e) {
    return e == hipErrorOutOfMemory ? SCFFT_ERR_OOM : SCFFT_ERR_DEVICE;
  };
  hipError_t e;
  if ((e = hipMalloc(&p->X, p->xbytes)) != hipSuccess) return fail(e);
  if ((e = hipMalloc(&p->Ep, p->rbytes)) != hipSuccess) return fail(e);
  if (p->st) {
    if ((e = hipMalloc(&p->S, p->rbytes)) != hipSuccess) return fail(e);
    if ((e = hipMalloc(&p->T, p->rbytes)) != hipSuccess) return fail(e);
  }
  const size_t pb = (size_t)std::max(part_blocks, p->xblocks);
  if ((e = hipMalloc(&p->part, sizeof(double) * 5 * (size_t)nsolve * d * pb)) != hipSuccess)
    return fail(e);
  if ((e = hipMalloc(&p->ctl, sizeof(SolveCtl) * nsolve)) != hipSuccess) return fail(e);
  if ((e = hipMalloc(&p->coef, sizeof(SolveCoef) * nsolve)) != hipSuccess) return fail(e);
  for (int a = 0; a < d; ++a) {
    if ((e = hipMalloc(&p->tw[a], p->esz * p->n[a])) != hipSuccess) return fail(e);
    if ((e = hipMalloc(&p->sym[a], 2 * sizeof(double) * p->n[a])) != hipSuccess) return fail(e);
  }
  scfft_status rc = plan_tables(p, stream);
  if (rc != SCFFT_OK) return rc;
  return ensure_hist(p, 64);
}

// ---------------------------------------------------------------- autotuner
// One solve's configuration, used to time candidate knobs on the real kernels.
struct TuneCtx {
  int mk;
  const SolveCtl* ctl;
  const SolveCoef* coef;
  const uint8_t* phase;
  const double* density;
};

using TuneKey = std::tuple<int, int, int, int, int, int, bool, int, bool, int>;
std::map<TuneKey, Knobs> g_tuned;
bool g_tune_file_read = false;

bool tuning_enabled() { return env_int("SCFFT_TUNE", 1) != 0; }

std::string arch_name(int dev) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  return a.substr(0, a.find(':'));
}

// On-disk cache (SCFFT_TUNE_CACHE): one line per tuned configuration,
// "arch d n0 n1 n2 prec st symbol real mk xr gr gC yC pack nt pitch".
void tune_file_read(int dev) {
  if (g_tune_file_read) return;
  g_tune_file_read = true;
  const char* path = std::getenv("SCFFT_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  const std::string arch = arch_name(dev);
  char a[64];
  int v[16];
  while (std::fscanf(f, "%63s %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d", a, &v[0], &v[1],
                     &v[2], &v[3], &v[4], &v[5], &v[6], &v[7], &v[8], &v[9], &v[10], &v[11],
                     &v[12], &v[13], &v[14], &v[15]) == 17) {
    if (arch != a) continue;
    Knobs k;
    k.xr = v[9];
    k.gr = v[10];
    k.gC = v[11];
    k.yC = v[12];
    k.pack = v[13];
    k.nt = v[14];
    k.pitch = v[15];
    g_tuned[TuneKey{dev, v[0], v[1], v[2], v[3], v[4], v[5] != 0, v[6], v[7] != 0, v[8]}] = k;
  }
  std::fclose(f);
}

void tune_file_append(const TuneKey& t, const Knobs& k) {
  const char* path = std::getenv("SCFFT_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d\n",
               arch_name(std::get<0>(t)).c_str(), std::get<1>(t), std::get<2>(t), std::get<3>(t),
               std::get<4>(t), std::get<5>(t), (int)std::get<6>(t), std::get<7>(t),
               (int)std::get<8>(t), std::get<9>(t), k.xr, k.gr, k.gC, k.yC, k.pack, k.nt, k.pitch);
  std::fclose(f);
}

scfft_status launch_iteration(Plan* p, const uint8_t* phase, const double* density, hipStream_t st,
                              bool ignore_done, hipEvent_t* ev);
scfft_status launch_init(Plan* p, hipStream_t st);

// Sets the per-pass knobs of a shaped plan in place (same buffer layout).
void set_pass_knobs(Plan* p, int xr, int gr, int gC, int yC) {
  const int esz = (int)p->esz;
  if (p->p2x && xr) {
    p->kn.xr = xr;
    p->xL = xpass_lines(p->n[0], esz, xr);
    p->xblocks = p->real ? (p->xlines / 2 + p->xL - 1) / p->xL : (p->xlines + p->xL - 1) / p->xL;
  }
  if (gr) p->kn.gr = gr;
  if (gC) p->kn.gC = p->gC = gC;
  if (yC) p->kn.yC = p->yC = yC;
}

// Times every candidate of each pass on scratch plans of every layout
// (pack / pitch / nontemporal streams) with the solve's own coefficients:
// per candidate one untimed and three timed iterations, the fastest of the
// three per pass.  Within a layout the passes are independent, so the i-th
// candidates of all passes run together; a layout costs the sum of its
// fastest passes (the y pass twice in 3D); the cheapest layout wins.
scfft_status autotune(int dev, int d, const int* n, int prec, bool st, int symbol, bool real,
                      const TuneCtx& tc, hipStream_t stream, Knobs* out) {
  Plan probe;
  plan_shape(&probe, dev, d, n, prec, 1, st, symbol, real);
  const int esz = (int)probe.esz;
  const int nlast = n[d - 1];
  std::vector<int> xrs = probe.p2x ? std::vector<int>{4, 8} : std::vector<int>{0};
  std::vector<std::pair<int, int>> gcs;   // (radix, tile width)
  if (probe.p2g) {
    std::vector<int> radices{4, 8};
    if (d == 2 && nlast == 2048 && esz == 16) radices.push_back(16);
    for (int r : radices) {
      if (nlast < r) continue;
      const int cmax = line_tile_max(nlast, esz, d, r);
      if (r == 16) {
        gcs.push_back({r, cmax});
        continue;
      }
      for (int c = 1; c <= std::min(cmax, 8); c *= 2) gcs.push_back({r, c});
    }
  } else if (probe.smg) {
    gcs.push_back({0, probe.gC});
  } else {
    const int el = elems_for(prec);
    const int cmax = std::min(pow2_floor(std::max(1, el / (nlast * d))), n[0]);
    for (int c = 1; c <= std::min(cmax, 8); c *= 2) gcs.push_back({0, c});
  }
  std::vector<int> ycs{0};
  if (d == 3) {
    ycs.clear();
    const int el = elems_for(prec);
    const int cmax = probe.p2y ? line_tile_max(n[1], esz, 1, 8)
                               : std::min(pow2_floor(std::max(1, el / n[1])), n[0]);
    if (probe.smy) ycs.push_back(probe.yC);
    else
      for (int c = 1; c <= std::min(cmax, 8); c *= 2) ycs.push_back(c);
  }
  const std::vector<int> packs = (real && d == 2 && probe.p2g && probe.p2x)
                                     ? std::vector<int>{0, 1} : std::vector<int>{0};
  const std::vector<int> bins = real ? std::vector<int>{0, 1} : std::vector<int>{0};
  // nontemporal streams: the register real-field x pass only
  const std::vector<int> nts = (real && !probe.smx) ? std::vector<int>{0, 1} : std::vector<int>{0};
  int part_blocks = 0;
  for (int xr : xrs) {
    Plan t = probe;
    set_pass_knobs(&t, xr, 0, 0, 0);
    part_blocks = std::max(part_blocks, t.xblocks);
  }
  hipEvent_t ev[10];
  for (auto& e : ev) SCFFT_HIP(hipEventCreate(&e));
  double best_cost = INFINITY;
  Knobs best = probe.kn;
  scfft_status rc = SCFFT_OK;
  const size_t rounds = std::max({xrs.size(), gcs.size(), ycs.size()});
  for (int pack : packs)
    for (int pitch : bins)
      for (int nt : nts) {
        if (rc != SCFFT_OK) break;
        Knobs lay;
        lay.pack = pack;
        lay.pitch = pitch;
        lay.nt = nt;
        lay.xr = xrs[0];
        lay.gr = gcs[0].first;
        lay.gC = gcs[0].second;
        lay.yC = ycs[0];
        Plan* p = new Plan();
        plan_shape(p, dev, d, n, prec, 1, st, symbol, real, lay);
        if (p->kn.pack != pack || p->kn.pitch != pitch || p->kn.nt != nt) {
          free_plan(p);   // the environment forces this layout knob: nothing to time
          continue;
        }
        rc = plan_alloc(p, stream, part_blocks);
        if (rc == SCFFT_OK) {
          p->mk = tc.mk;
          if (hipMemcpyAsync(p->ctl, tc.ctl, sizeof(SolveCtl), hipMemcpyHostToDevice, stream) !=
                  hipSuccess ||
              hipMemcpyAsync(p->coef, tc.coef, sizeof(SolveCoef), hipMemcpyHostToDevice,
                             stream) != hipSuccess)
            rc = SCFFT_ERR_DEVICE;
        }
        if (rc == SCFFT_OK) rc = launch_init(p, stream);
        std::vector<double> tx(xrs.size(), INFINITY), tg(gcs.size(), INFINITY),
            ty(ycs.size(), INFINITY);
        for (size_t i = 0; i < rounds && rc == SCFFT_OK; ++i) {
          const size_t ix = i % xrs.size(), ig = i % gcs.size(), iy = i % ycs.size();
          set_pass_knobs(p, xrs[ix], gcs[ig].first, gcs[ig].second, ycs[iy]);
          for (int rep = 0; rep < 4 && rc == SCFFT_OK; ++rep) {
            rc = launch_iteration(p, tc.phase, tc.density, stream, true, ev);
            if (rc != SCFFT_OK) break;
            if (hipEventSynchronize(ev[d == 3 ? 9 : 7]) != hipSuccess) {
              rc = SCFFT_ERR_DEVICE;
              break;
            }
            if (rep == 0) continue;
            float a = 0, b = 0, c = 0, e2 = 0;
            (void)hipEventElapsedTime(&a, ev[0], ev[1]);
            (void)hipEventElapsedTime(&b, ev[6], ev[7]);
            if (d == 3) {
              (void)hipEventElapsedTime(&c, ev[4], ev[5]);
              (void)hipEventElapsedTime(&e2, ev[8], ev[9]);
            }
            tx[ix] = std::min(tx[ix], (double)a);
            tg[ig] = std::min(tg[ig], (double)b);
            ty[iy] = std::min(ty[iy], (double)(c + e2));
          }
        }
        if (rc == SCFFT_OK) {
          const size_t bx = std::min_element(tx.begin(), tx.end()) - tx.begin();
          const size_t bg = std::min_element(tg.begin(), tg.end()) - tg.begin();
          const size_t by = std::min_element(ty.begin(), ty.end()) - ty.begin();
          const double cost = tx[bx] + tg[bg] + (d == 3 ? ty[by] : 0.0);
          if (cost < best_cost) {
            best_cost = cost;
            best = lay;
            best.xr = xrs[bx];
            best.gr = gcs[bg].first;
            best.gC = gcs[bg].second;
            best.yC = ycs[by];
          }
        }
        (void)hipStreamSynchronize(stream);
        free_plan(p);
      }
  for (auto& e : ev) (void)hipEventDestroy(e);
  if (rc != SCFFT_OK) return rc;
  *out = best;
  return SCFFT_OK;
}

// Knobs for a configuration: the cached tuning (tuned on first use when a
// solve's configuration is given and tuning is on), else the rules.
scfft_status knobs_for(int dev, int d, const int* n, int prec, bool st, int symbol, bool real,
                       const TuneCtx* tc, hipStream_t stream, Knobs* out, bool* tuned) {
  *out = Knobs();
  *tuned = false;
  if (!tuning_enabled() || !tc) return SCFFT_OK;
  tune_file_read(dev);
  const int n2 = d == 3 ? n[2] : 1;
  const TuneKey key{dev, d, n[0], n[1], n2, prec, st, symbol, real, tc->mk};
  auto it = g_tuned.find(key);
  if (it == g_tuned.end()) {
    Knobs k;
    scfft_status rc = autotune(dev, d, n, prec, st, symbol, real, *tc, stream, &k);
    if (rc != SCFFT_OK) return rc;
    it = g_tuned.emplace(key, k).first;
    tune_file_append(key, k);
  }
  *out = it->second;
  *tuned = true;
  return SCFFT_OK;
}

// Knobs already tuned for a configuration (no tuning: for callers that may
// not allocate), else the rules.
Knobs cached_knobs(int dev, int d, const int* n, int prec, bool st, int symbol, bool real, int mk,
                   bool* tuned) {
  const int n2 = d == 3 ? n[2] : 1;
  auto it = g_tuned.find(TuneKey{dev, d, n[0], n[1], n2, prec, st, symbol, real, mk});
  *tuned = tuning_enabled() && it != g_tuned.end();
  return *tuned ? it->second : Knobs();
}

// `slot` separates workspaces of same-shaped problems solved together; tc
// (optional) is one solve's configuration for the autotuner.
scfft_status get_plan(int d, const int* n, int prec, int nsolve, bool st, int symbol,
                      hipStream_t stream, Plan** out, int slot = 0, bool real = false,
                      const TuneCtx* tc = nullptr) {
  int dev = 0;
  SCFFT_HIP(hipGetDevice(&dev));
  const int n2 = d == 3 ? n[2] : 1;
  PlanKey key{dev, d, n[0], n[1], n2, prec, nsolve, st, symbol, slot, real};
  auto it = g_plans.find(key);
  if (it != g_plans.end()) {
    *out = it->second;
    return SCFFT_OK;
  }
  Knobs want;
  bool tuned = false;
  scfft_status rc = knobs_for(dev, d, n, prec, st, symbol, real, tc, stream, &want, &tuned);
  if (rc != SCFFT_OK) return rc;
  Plan* p = new Plan();
  plan_shape(p, dev, d, n, prec, nsolve, st, symbol, real, want);
  p->tuned = tuned;
  rc = plan_alloc(p, stream);
  if (rc != SCFFT_OK) {
    free_plan(p);
    return rc;
  }
  g_plans[key] = p;
  *out = p;
  return SCFFT_OK;
}

// ------------------------------------------------------------- host scalars
void put(double* dst, cd v) {
  dst[0] = v.real();
  dst[1] = v.imag();
}

struct Scalars {
  cd sigma0, t, z, p[3], e2p, j3p;
};

// p from (alpha, beta): eq. J24 solved for p1^2, p2^2 with p^T p = 1.
void p_from_interval(double a, double b, cd* p) {
  const double w = b - a;
  p[0] = std::sqrt(cd((1 + a) * (1 + b) / w, 0));
  p[1] = std::sqrt(cd(-(1 + a) / w, 0));
  p[2] = std::sqrt(cd(-a * (1 + b) / w, 0));
}

// t(sigma1) of eq. J3 / J23.
cd t_map(cd s, double a, double b) { return (s + a) * (1.0 + b) / ((s + b) * (1.0 + a)); }

scfft_status scheme_scalars(int scheme, cd s1, double a, double b, Scalars* out) {
  Scalars r{};
  if (scheme == SCFFT_ACC_EM || scheme == SCFFT_ACC_MS) {
    if (!(a > 0.0 && b > a && std::isfinite(b))) return SCFFT_ERR_INVALID_ARG;
    if (s1.imag() == 0.0 && s1.real() >= -b && s1.real() <= -a) return SCFFT_ERR_SLIT;
    p_from_interval(a, b, r.p);
    r.t = t_map(s1, a, b);
    const cd w = std::sqrt(r.t);
    if (scheme == SCFFT_ACC_EM) {
      r.sigma0 = w;
      r.z = (w - 1.0) / (w + 1.0);
    } else {
      r.sigma0 = (r.t + 1.0) / 2.0;
      r.z = (r.t - 1.0) / (r.t + 1.0);
    }
    const cd den = (r.t - 1.0) * r.p[1] * r.p[1] + 1.0;
    r.e2p = (1.0 - r.t) * r.p[0] * r.p[1] / den;    // eq. J21
    r.j3p = r.p[0] * r.p[2] * (r.t - 1.0) / den;    // eq. J26
  } else if (scheme == SCFFT_MS) {
    r.sigma0 = (s1 + 1.0) / 2.0;
    r.z = (s1 - 1.0) / (s1 + 1.0);                   // eq. J1
  } else if (scheme == SCFFT_EM) {
    if (s1.imag() == 0.0 && s1.real() <= 0.0) return SCFFT_ERR_SLIT;
    r.sigma0 = std::sqrt(s1);
    r.z = (r.sigma0 - 1.0) / (r.sigma0 + 1.0);       // eq. J2
  } else {
    return SCFFT_ERR_INVALID_ARG;
  }
  *out = r;
  return SCFFT_OK;
}

// Fill the per-phase coefficient tables of a two-phase or graded medium.
void fill_local(SolveCoef& c, int kind, cd s1, cd s0) {
  const cd sig[2] = {cd(1, 0), s1};
  for (int ph = 0; ph < 2; ++ph) {
    const cd s = sig[ph];
    cd cE(1, 0), cO, cJ = s, cS(0, 0);
    if (kind == K_MS) {
      cO = 1.0 - s / s0;
    } else if (kind == K_EM) {
      cE = 1.0 / (s + s0);
      cO = (s - s0) / (s + s0);
    } else if (kind == K_ADJ) {
      cO = (s - s0) / (s + s0);
      cJ = 0.0;
      cS = s / (s + s0);
    }
    put(c.cE[ph], cE);
    put(c.cO[ph], cO);
    put(c.cJ[ph], cJ);
    put(c.cS[ph], cS);
  }
  put(c.s1, s1);
  put(c.s0, s0);
}

struct SolveSpec {
  int kind;
  cd s1, s0;
  Scalars sc;
  int power_phase;   // K_POWER: weight chi (1) or 1 - chi (0)
};

void fill_coef(SolveCoef& c, const SolveSpec& sp, bool density, int d, const double* e0, double M) {
  std::memset(&c, 0, sizeof(c));
  c.kind = sp.kind;
  c.density = density ? 1 : 0;
  cd src(0, 0), init(0, 0);   // multipliers of e0
  switch (sp.kind) {
    case K_MS:
      fill_local(c, K_MS, sp.s1, sp.s0);
      c.ga = 0;
      c.gb = 1;
      c.kz_keep = 0;
      src = init = 1.0;
      break;
    case K_EM:
      fill_local(c, K_EM, sp.s1, sp.s0);
      c.ga = 1;
      c.gb = -2;
      c.kz_keep = 1;
      src = init = 2.0 * sp.s0;
      break;
    case K_ADJ:
      fill_local(c, K_ADJ, sp.s1, sp.s0);
      c.ga = 1;
      c.gb = -2;
      c.kz_keep = 1;
      break;
    case K_POWER: {
      for (int ph = 0; ph < 2; ++ph) {
        const double w = (ph == sp.power_phase) ? 1.0 : 0.0;
        put(c.cE[ph], 1.0);
        put(c.cO[ph], w);
        put(c.cJ[ph], w);
        put(c.cS[ph], 0.0);
      }
      c.ga = 0;
      c.gb = 1;
      c.kz_keep = 0;
      init = 1.0;
      break;
    }
    case K_ACC_EM:
    case K_ACC_MS: {
      put(c.s1, sp.s1);
      put(c.s0, sp.s0);
      for (int i = 0; i < 3; ++i) put(c.p[i], sp.sc.p[i]);
      put(c.z, sp.sc.z);
      const cd w = std::sqrt(sp.sc.t);
      put(c.inv1w, 1.0 / (1.0 + w));
      put(c.p1kap, sp.sc.p[0] * (1.0 / (sp.sc.t + w) - 1.0 / (1.0 + w)));
      if (sp.kind == K_ACC_EM) {
        c.ga = 1;
        c.gb = -2;
        c.kz_keep = 1;
        src = init = 2.0 * w;
      } else {
        c.ga = 0;
        c.gb = 1;
        c.kz_keep = 0;
        src = init = 1.0;
      }
      break;
    }
  }
  for (int i = 0; i < d; ++i) {
    put(c.kz_src[i], src * (M * e0[i]));
    put(c.init_src[i], init * (M * e0[i]));
  }
}

void fill_ctl(SolveCtl& c, const scfft_options& o, int kind, int d, const double* e0) {
  std::memset(&c, 0, sizeof(c));
  c.tol = o.tol;
  c.div_factor = o.div_factor;
  c.max_iter = o.max_iter;
  c.stag_window = o.stag_window;
  double n2 = 0;
  for (int i = 0; i < d; ++i) {
    c.e0[i] = e0[i];
    n2 += e0[i] * e0[i];
  }
  c.inv_e0n2 = 1.0 / n2;
  c.d = d;
  c.kind = kind;
}

// ------------------------------------------------------------------ launches
template <typename T>
scfft_status launch_iteration_t(Plan* p, const uint8_t* phase, const double* density,
                                hipStream_t st, bool ignore_done, hipEvent_t* ev) {
  const int d = p->d;
  const size_t esz = sizeof(cx<T>);
  auto rec = [&](int k) {
    if (ev) (void)hipEventRecord(ev[k], st);
  };
  {
    XArgs a{};
    a.X = p->X;
    a.Eprev = p->Ep;
    a.Sslot = p->S;
    a.Tslot = p->T;
    a.phase = phase;
    a.density = density;
    a.part = p->part;
    a.ctl = p->ctl;
    a.coef = p->coef;
    a.tw = p->tw[0];
    a.fd = p->fd[0];
    a.M = p->M;
    a.Mh = p->Mh;
    a.hp = p->HP;
    a.n0 = p->n[0];
    a.nlines = p->xlines;
    a.lines_per_block = p->xL;
    a.d = d;
    a.invM = 1.0 / (double)p->M;
    a.ignore_done = ignore_done;
    a.packed = p->packed ? 1 : 0;
    // the x pass reuses its LDS for a 5 x (kNT/64) fp64 reduction
    rec(0);
    const dim3 grid(p->xblocks, d, p->nsolve);
    if (p->real && p->smx) {
      if (!launch_xpass_smooth_real<T>(a, grid, st, p->n[0], p->mk)) return SCFFT_ERR_DEVICE;
    } else if (p->real) {
      launch_xpass_real<T>(a, grid, st, p->n[0], p->mk, p->nt, p->kn.xr);
    } else if (p->p2x) {
      launch_xpass_reg<T>(a, grid, st, p->n[0], p->mk, p->kn.xr);
    } else if (p->smx) {
      if (!launch_xpass_smooth<T>(a, grid, st, p->n[0], p->mk)) return SCFFT_ERR_DEVICE;
    } else {
      const size_t lds =
          std::max((size_t)p->xL * p->n[0] * esz, (size_t)5 * (kNT / 64) * sizeof(double));
      launch_xpass_generic<T>(a, grid, lds, st);
    }
    rec(1);
  }
  FArgs f{};
  f.part = p->part;
  f.ctl = p->ctl;
  f.hist_r = p->hist_r;
  f.hist_s = p->hist_s;
  f.hist_cap = p->hist_cap;
  f.nblocks = p->xblocks;
  f.invM = 1.0 / (double)p->M;
  f.ignore_done = ignore_done;
  rec(2);
  rec(3);
  GArgs g{};
  g.X = p->X;
  g.ctl = p->ctl;
  g.coef = p->coef;
  g.M = p->Mh;
  g.n[0] = p->H;   // columns of X (n0, or n0/2 + 1 in real mode)
  g.n[1] = p->n[1];
  g.n[2] = p->n[2];
  g.d = d;
  g.symbol = p->symbol;
  g.ignore_done = ignore_done;
  g.f = f;
  g.fin = 0;
  g.packed = p->packed ? 1 : 0;
  g.rp = p->HP;
  for (int a = 0; a < d; ++a) g.symtab[a] = p->sym[a];
  if (d == 3) {
    GArgs y = g;
    y.tw = p->tw[1];
    y.fd = p->fd[1];
    y.C = p->yC;
    y.stride = p->HP;
    y.mode = 1;
    y.fin = 0;   // the stop rules run in the Gamma pass (measured cheaper there)
    dim3 grid((p->H + p->yC - 1) / p->yC, p->n[2], p->nsolve * d);
    rec(4);
    if (p->p2y) {
      launch_line_reg<T, 1>(y, grid, st, p->n[1], 8);
    } else if (p->smy) {
      if (!launch_ypass_smooth<T>(y, grid, st, p->n[1])) return SCFFT_ERR_DEVICE;
    } else {
      launch_line_generic<T>(y, grid, (size_t)p->n[1] * p->yC * esz, st);
    }
    rec(5);
  }
  {
    GArgs q = g;
    const int nl = p->n[d - 1];
    q.tw = p->tw[d - 1];
    q.fd = p->fd[d - 1];
    q.C = p->gC;
    q.stride = d == 2 ? p->HP : p->HP * p->n[1];
    q.mode = 0;
    q.fin = 1;
    dim3 grid((p->H + p->gC - 1) / p->gC, d == 3 ? p->n[1] : 1, p->nsolve);
    if (p->p2g && q.fin) grid.x += 1;   // the finalizing workgroups
    rec(6);
    if (p->p2g && p->kn.gr == 16) {
      if constexpr (sizeof(T) == 8) launch_line_r16_f64_2048(q, grid, st);
    } else if (p->p2g) {
      if (d == 2) launch_line_reg<T, 2>(q, grid, st, nl, p->kn.gr);
      else launch_line_reg<T, 3>(q, grid, st, nl, p->kn.gr);
    } else if (p->smg) {
      if (!launch_gamma_smooth<T>(q, grid, st, nl, d)) return SCFFT_ERR_DEVICE;
    } else {
      launch_line_generic<T>(q, grid, (size_t)nl * d * p->gC * esz, st);
    }
    rec(7);
  }
  if (d == 3) {
    GArgs y = g;
    y.tw = p->tw[1];
    y.fd = p->fd[1];
    y.C = p->yC;
    y.stride = p->HP;
    y.mode = 2;
    const dim3 grid((p->H + p->yC - 1) / p->yC, p->n[2], p->nsolve * d);
    rec(8);
    if (p->p2y) {
      launch_line_reg<T, 1>(y, grid, st, p->n[1], 8);
    } else if (p->smy) {
      if (!launch_ypass_smooth<T>(y, grid, st, p->n[1])) return SCFFT_ERR_DEVICE;
    } else {
      launch_line_generic<T>(y, grid, (size_t)p->n[1] * p->yC * esz, st);
    }
    rec(9);
  }
  SCFFT_HIP(hipGetLastError());
  return SCFFT_OK;
}

scfft_status launch_iteration(Plan* p, const uint8_t* phase, const double* density, hipStream_t st,
                              bool ignore_done = false, hipEvent_t* ev = nullptr) {
  if (p->prec == SCFFT_FP32)
    return launch_iteration_t<float>(p, phase, density, st, ignore_done, ev);
  return launch_iteration_t<double>(p, phase, density, st, ignore_done, ev);
}

scfft_status launch_init(Plan* p, hipStream_t st) {
  if (p->nsolve > 256) return SCFFT_ERR_INVALID_ARG;
  if (p->real) {
    InitRArgs r{};
    r.X = p->X;
    r.Sslot = p->S;
    r.Tslot = p->T;
    r.ctl = p->ctl;
    r.coef = p->coef;
    r.M = p->M;
    r.Mh = p->Mh;
    r.d = p->d;
    r.H = p->HP;
    r.nsolve = p->nsolve;
    r.has_st = p->st ? 1 : 0;
    const long long tot = (long long)p->nsolve * p->d * p->M;
    const int blocks = (int)std::min<long long>((tot + 255) / 256, 65536);
    if (p->prec == SCFFT_FP32)
      hipLaunchKernelGGL(init_real_kernel<float>, dim3(blocks), dim3(256), 0, st, r);
    else
      hipLaunchKernelGGL(init_real_kernel<double>, dim3(blocks), dim3(256), 0, st, r);
    SCFFT_HIP(hipGetLastError());
    return SCFFT_OK;
  }
  InitArgs a{};
  a.X = p->X;
  a.Sslot = p->S;
  a.Tslot = p->T;
  a.ctl = p->ctl;
  a.coef = p->coef;
  a.M = p->M;
  a.d = p->d;
  a.n0 = p->n[0];
  a.nsolve = p->nsolve;
  a.has_st = p->st ? 1 : 0;
  a.src_scale = (double)p->M;
  const long long tot = (long long)p->nsolve * p->d * p->M;
  const int blocks = (int)std::min<long long>((tot + 255) / 256, 65536);
  if (p->nsolve > 256) return SCFFT_ERR_INVALID_ARG;
  if (p->prec == SCFFT_FP32)
    hipLaunchKernelGGL(init_kernel<float>, dim3(blocks), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(init_kernel<double>, dim3(blocks), dim3(256), 0, st, a);
  SCFFT_HIP(hipGetLastError());
  return SCFFT_OK;
}

scfft_status launch_extract(Plan* p, int solve, const uint8_t* phase, const double* density,
                            scfft_c64* E, scfft_c64* J, hipStream_t st) {
  if (!E && !J) return SCFFT_OK;
  ExtractArgs a{};
  a.Eprev = p->Ep;
  a.phase = phase;
  a.density = density;
  a.coef = p->coef;
  a.E = reinterpret_cast<double*>(E);
  a.J = reinterpret_cast<double*>(J);
  a.M = p->M;
  a.d = p->d;
  a.solve = solve;
  const long long tot = (long long)p->d * p->M;
  const int blocks = (int)std::min<long long>((tot + 255) / 256, 65536);
  if (p->real) {
    if (p->prec == SCFFT_FP32)
      hipLaunchKernelGGL(extract_real_kernel<float>, dim3(blocks), dim3(256), 0, st, a);
    else
      hipLaunchKernelGGL(extract_real_kernel<double>, dim3(blocks), dim3(256), 0, st, a);
  } else if (p->prec == SCFFT_FP32) {
    hipLaunchKernelGGL(extract_kernel<float>, dim3(blocks), dim3(256), 0, st, a);
  } else {
    hipLaunchKernelGGL(extract_kernel<double>, dim3(blocks), dim3(256), 0, st, a);
  }
  SCFFT_HIP(hipGetLastError());
  return SCFFT_OK;
}

// ----------------------------------------------------------- graph cache
// One chunk of check_every iterations over all plans is captured into a HIP
// graph and replayed until every solve has stopped.  Kernel arguments do not
// change between iterations (the iteration state lives in device memory), so
// a captured chunk stays valid for every later solve on the same plans and
// input pointers; the key records everything the arguments depend on.
struct GraphEntry {
  std::vector<uintptr_t> key;
  hipGraphExec_t exec = nullptr;
};
std::vector<GraphEntry> g_graphs;
std::map<int, hipStream_t> g_work_streams;

void free_graphs() {
  for (auto& g : g_graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  g_graphs.clear();
}

// Drops the oldest cached graphs beyond `keep`.  Called only before a loop
// gathers its graphs, so no handle a running loop holds is destroyed.
void trim_graphs(size_t keep) {
  while (g_graphs.size() > keep) {
    (void)hipGraphExecDestroy(g_graphs.front().exec);
    g_graphs.erase(g_graphs.begin());
  }
}

// Graph capture needs a stream other than the legacy default stream.
// Per device: the loop's two timing events and the event that orders the
// work stream after the caller's stream (created once).
struct LoopEvents {
  hipEvent_t t0, t1, dep;
};
std::map<int, LoopEvents> g_loop_events;

scfft_status loop_events(LoopEvents* out) {
  int dev = 0;
  SCFFT_HIP(hipGetDevice(&dev));
  auto it = g_loop_events.find(dev);
  if (it == g_loop_events.end()) {
    LoopEvents e{};
    SCFFT_HIP(hipEventCreate(&e.t0));
    SCFFT_HIP(hipEventCreate(&e.t1));
    SCFFT_HIP(hipEventCreateWithFlags(&e.dep, hipEventDisableTiming));
    it = g_loop_events.emplace(dev, e).first;
  }
  *out = it->second;
  return SCFFT_OK;
}

scfft_status work_stream(hipStream_t st, hipStream_t* ws) {
  if (st != nullptr) {
    *ws = st;
    return SCFFT_OK;
  }
  int dev = 0;
  SCFFT_HIP(hipGetDevice(&dev));
  auto it = g_work_streams.find(dev);
  if (it == g_work_streams.end()) {
    hipStream_t s;
    SCFFT_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    it = g_work_streams.emplace(dev, s).first;
  }
  *ws = it->second;
  return SCFFT_OK;
}

// Streams (default priority) and events that fork and join the parallel
// branches of a captured batch graph, one set per device.
constexpr int kBranches = 4;
struct Branches {
  hipStream_t s[kBranches];
  hipEvent_t fork;
  hipEvent_t join[kBranches];
};
std::map<int, Branches> g_branches;

scfft_status branches_for(int dev, Branches** out) {
  auto it = g_branches.find(dev);
  if (it == g_branches.end()) {
    Branches b{};
    for (int i = 0; i < kBranches; ++i) {
      SCFFT_HIP(hipStreamCreateWithFlags(&b.s[i], hipStreamNonBlocking));
      SCFFT_HIP(hipEventCreateWithFlags(&b.join[i], hipEventDisableTiming));
    }
    SCFFT_HIP(hipEventCreateWithFlags(&b.fork, hipEventDisableTiming));
    it = g_branches.emplace(dev, b).first;
  }
  *out = &it->second;
  return SCFFT_OK;
}

scfft_status get_graph(const std::vector<Plan*>& plans, const std::vector<const uint8_t*>& phases,
                       const std::vector<const double*>& dens, int ce, hipStream_t ws,
                       hipGraphExec_t* out) {
  std::vector<uintptr_t> key = {(uintptr_t)ws, (uintptr_t)ce};
  for (size_t i = 0; i < plans.size(); ++i) {
    key.push_back((uintptr_t)plans[i]);
    key.push_back((uintptr_t)plans[i]->mk);
    key.push_back((uintptr_t)plans[i]->hist_r);
    key.push_back((uintptr_t)plans[i]->hist_cap);
    key.push_back((uintptr_t)phases[i]);
    key.push_back((uintptr_t)dens[i]);
  }
  for (auto& g : g_graphs)
    if (g.key == key) {
      *out = g.exec;
      return SCFFT_OK;
    }
  // Several plans (a batch of structures) become parallel branches of the
  // graph, at most kBranches, each a chain of its plans' iterations; plans
  // go to the least loaded branch, largest first (cost: voxels x solves).
  const int nbmax = std::max(1, std::min(kBranches, env_int("SCFFT_BRANCHES", kBranches)));
  const int nb = (int)std::min<size_t>(plans.size(), (size_t)nbmax);
  std::vector<int> branch(plans.size(), 0);
  if (nb > 1) {
    std::vector<size_t> order(plans.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](size_t a, size_t b) {
      return plans[a]->M * plans[a]->nsolve > plans[b]->M * plans[b]->nsolve;
    });
    std::vector<long long> load(nb, 0);
    for (size_t i : order) {
      const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      branch[i] = b;
      load[b] += plans[i]->M * plans[i]->nsolve;
    }
  }
  Branches* br = nullptr;
  if (nb > 1) {
    scfft_status rb = branches_for(plans[0]->dev, &br);
    if (rb != SCFFT_OK) return rb;
  }
  SCFFT_HIP(hipStreamBeginCapture(ws, hipStreamCaptureModeThreadLocal));
  scfft_status rc = SCFFT_OK;
  if (nb > 1) {
    if (hipEventRecord(br->fork, ws) != hipSuccess) rc = SCFFT_ERR_DEVICE;
    for (int b = 0; b < nb && rc == SCFFT_OK; ++b)
      if (hipStreamWaitEvent(br->s[b], br->fork, 0) != hipSuccess) rc = SCFFT_ERR_DEVICE;
  }
  for (int k = 0; k < ce && rc == SCFFT_OK; ++k)
    for (size_t i = 0; i < plans.size() && rc == SCFFT_OK; ++i)
      rc = launch_iteration(plans[i], phases[i], dens[i], nb > 1 ? br->s[branch[i]] : ws);
  if (nb > 1)
    for (int b = 0; b < nb && rc == SCFFT_OK; ++b)
      if (hipEventRecord(br->join[b], br->s[b]) != hipSuccess ||
          hipStreamWaitEvent(ws, br->join[b], 0) != hipSuccess)
        rc = SCFFT_ERR_DEVICE;
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(ws, &graph);
  if (rc != SCFFT_OK || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc != SCFFT_OK ? rc : SCFFT_ERR_DEVICE;
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e2 != hipSuccess) return SCFFT_ERR_DEVICE;
  // upload now, so that the first replay (perhaps inside a caller's timed
  // region) does not pay for it
  if (hipGraphUpload(exec, ws) != hipSuccess) {
    (void)hipGraphExecDestroy(exec);
    return SCFFT_ERR_DEVICE;
  }
  g_graphs.push_back(GraphEntry{key, exec});
  *out = exec;
  return SCFFT_OK;
}

// Iterate every solve of the given plans until all have stopped.  Work made
// earlier on `st` must be complete or ordered before the loop (callers
// synchronise after their set-up copies).
scfft_status run_loop(const std::vector<Plan*>& plans, const std::vector<const uint8_t*>& phases,
                      const std::vector<const double*>& dens, int max_iter, int check_every,
                      hipStream_t st, double* elapsed_ms, bool allow_graph = true,
                      hipEvent_t* timing = nullptr,
                      std::vector<std::vector<SolveCtl>>* final_ctl = nullptr) {
  // a solve shorter than one check interval runs as a single chunk
  const int ce = std::max(1, std::min(check_every, max_iter + 1));
  const bool use_graph = allow_graph && !std::getenv("SCFFT_NO_GRAPH");
  // the loop's own events, when it needs any (a caller that brings its
  // timing events and runs without graphs creates none)
  LoopEvents lev{};
  if (!timing || use_graph) {
    scfft_status rc = loop_events(&lev);
    if (rc != SCFFT_OK) return rc;
  }
  hipStream_t ws = st;
  if (use_graph) {
    scfft_status rc = work_stream(st, &ws);
    if (rc != SCFFT_OK) return rc;
    if (ws != st) {
      // the caller's set-up work on st comes first
      SCFFT_HIP(hipEventRecord(lev.dep, st));
      SCFFT_HIP(hipStreamWaitEvent(ws, lev.dep, 0));
    }
  }
  // A chunk of k iterations (k = ce, or what is left before max_iter, so no
  // launch beyond the last possible iterate is queued) replays graphs of 2^b
  // iterations: the largest (at most 64) as often as it fits, then one per
  // remaining set bit of k.  The graphs of every power of two up to
  // min(check_every, 64) are built at once on first use, so later solves of
  // any length build none.
  std::vector<hipGraphExec_t> pw;
  if (use_graph) {
    trim_graphs(192);
    for (int b = 0; (1 << b) <= std::min(std::max(1, check_every), 64); ++b) {
      hipGraphExec_t g = nullptr;
      scfft_status rc = get_graph(plans, phases, dens, 1 << b, ws, &g);
      if (rc != SCFFT_OK) return rc;
      pw.push_back(g);
    }
  }
  // timing events: the caller's or the loop's own
  const hipEvent_t e0 = timing ? timing[0] : lev.t0;
  const hipEvent_t e1 = timing ? timing[1] : lev.t1;
  SCFFT_HIP(hipEventRecord(e0, ws));
  // iterate n = 0..max_iter takes max_iter + 1 launches; a few spare chunks
  // cover solves whose stop flag is set by the last of them
  const long long max_chunks = (long long)(max_iter + 1) / ce + 3;
  const long long needed = (long long)max_iter + 1;
  long long launched = 0;
  std::vector<std::vector<SolveCtl>> host(plans.size());
  bool all_done = false;
  for (long long chunk = 0; chunk < max_chunks && !all_done; ++chunk) {
    const long long left = needed - launched;
    const int k = (int)(left >= ce || left <= 0 ? ce : left);
    if (use_graph) {
      const int top = (int)pw.size() - 1;
      int rem = k;
      for (; rem >= (1 << top); rem -= 1 << top) SCFFT_HIP(hipGraphLaunch(pw[top], ws));
      for (int b = top - 1; b >= 0; --b)
        if (rem & (1 << b)) SCFFT_HIP(hipGraphLaunch(pw[b], ws));
    } else {
      for (int q = 0; q < k; ++q)
        for (size_t i = 0; i < plans.size(); ++i) {
          scfft_status rc = launch_iteration(plans[i], phases[i], dens[i], ws);
          if (rc != SCFFT_OK) return rc;
        }
    }
    launched += k;
    all_done = true;
    // the loop's time ends with the last chunk's launches, before its read
    SCFFT_HIP(hipEventRecord(e1, ws));
    for (size_t i = 0; i < plans.size(); ++i) {
      Plan* q = plans[i];
      host[i].resize(q->nsolve);
      if (!q->no_alloc && !q->ctl_host)
        SCFFT_HIP(hipHostMalloc((void**)&q->ctl_host, sizeof(SolveCtl) * q->nsolve));
      SCFFT_HIP(hipMemcpyAsync(q->ctl_host ? (void*)q->ctl_host : (void*)host[i].data(), q->ctl,
                               sizeof(SolveCtl) * q->nsolve, hipMemcpyDeviceToHost, ws));
    }
    SCFFT_HIP(hipStreamSynchronize(ws));
    for (size_t i = 0; i < plans.size(); ++i)
      if (plans[i]->ctl_host)
        std::memcpy(host[i].data(), plans[i]->ctl_host, sizeof(SolveCtl) * plans[i]->nsolve);
    for (size_t i = 0; i < plans.size() && all_done; ++i)
      for (const auto& c : host[i])
        if (!c.done) {
          all_done = false;
          break;
        }
  }
  SCFFT_HIP(hipEventSynchronize(e1));   // complete already: the stream was synchronised
  float ms = 0;
  SCFFT_HIP(hipEventElapsedTime(&ms, e0, e1));
  if (elapsed_ms) *elapsed_ms = ms;
  if (!all_done) return SCFFT_ERR_DEVICE;   // the device never set its stop flag
  // the last check read every solve's final control block
  if (final_ctl) *final_ctl = std::move(host);
  return SCFFT_OK;
}

// `known`: the solve's final control block if the caller already has it
// (from the loop's last check); then a result without fields or histories
// needs no device access.
scfft_status read_result(Plan* p, int solve, const scfft_problem* prob, scfft_result* res,
                         hipStream_t st, double elapsed, const SolveCtl* known = nullptr) {
  SolveCtl c;
  const bool hist = res->history_cap > 0 && (res->residual_history || res->sigma_history);
  const bool device = !known || res->E || res->J || hist;
  if (known) c = *known;
  else SCFFT_HIP(hipMemcpyAsync(&c, p->ctl + solve, sizeof(SolveCtl), hipMemcpyDeviceToHost, st));
  scfft_status rc = launch_extract(p, solve, prob->phase, prob->density, res->E, res->J, st);
  if (rc != SCFFT_OK) return rc;
  const int n = c.iter;
  if (hist) {
    const int cnt = std::min(std::min(res->history_cap, n + 1), p->hist_cap);
    if (res->residual_history)
      SCFFT_HIP(hipMemcpyAsync(res->residual_history, p->hist_r + (size_t)solve * p->hist_cap,
                               sizeof(double) * cnt, hipMemcpyDeviceToHost, st));
    if (res->sigma_history)
      SCFFT_HIP(hipMemcpyAsync(res->sigma_history, p->hist_s + (size_t)solve * p->hist_cap * 2,
                               2 * sizeof(double) * cnt, hipMemcpyDeviceToHost, st));
  }
  if (device) SCFFT_HIP(hipStreamSynchronize(st));
  res->sigma_star.re = c.sstar_re;
  res->sigma_star.im = c.sstar_im;
  for (int i = 0; i < 3; ++i) {
    res->mean_J[i].re = i < p->d ? c.meanJ[2 * i] : 0.0;
    res->mean_J[i].im = i < p->d ? c.meanJ[2 * i + 1] : 0.0;
  }
  res->iterations = n;
  res->residual = c.res;
  res->status = c.status;
  res->elapsed_ms = elapsed;
  return (scfft_status)c.status;
}

long long voxels(const scfft_problem* p) {
  return (long long)p->n[0] * p->n[1] * (p->d == 3 ? p->n[2] : 1);
}

bool bad_e0(const scfft_problem* p) {
  double n2 = 0;
  for (int i = 0; i < p->d; ++i) {
    if (!std::isfinite(p->e0[i])) return true;
    n2 += p->e0[i] * p->e0[i];
  }
  return !(n2 > 0);
}

// Validates a problem/options pair and builds the solve spec.
scfft_status prepare(const scfft_problem* prob, const scfft_options* opt, cd s1, SolveSpec* sp) {
  if (!prob || !opt) return SCFFT_ERR_INVALID_ARG;
  scfft_status rc = check_dims(prob->d, prob->n, opt->precision);
  if (rc != SCFFT_OK) return rc;
  if (opt->precision != SCFFT_FP32 && opt->precision != SCFFT_FP64) return SCFFT_ERR_INVALID_ARG;
  if (opt->symbol < 0 || opt->symbol > 2) return SCFFT_ERR_INVALID_ARG;
  if (!prob->phase && !prob->density) return SCFFT_ERR_INVALID_ARG;
  if (bad_e0(prob) || opt->max_iter < 0 || std::isnan(opt->tol)) return SCFFT_ERR_INVALID_ARG;
  if (!std::isfinite(s1.real()) || !std::isfinite(s1.imag())) return SCFFT_ERR_INVALID_ARG;
  const bool acc = opt->scheme == SCFFT_ACC_EM || opt->scheme == SCFFT_ACC_MS;
  if (acc && prob->density) return SCFFT_ERR_INVALID_ARG;
  Scalars sc{};
  rc = scheme_scalars(opt->scheme, s1, opt->alpha, opt->beta, &sc);
  if (rc != SCFFT_OK) return rc;
  sp->s1 = s1;
  sp->sc = sc;
  sp->power_phase = 1;
  if (opt->scheme == SCFFT_MS) sp->kind = K_MS;
  else if (opt->scheme == SCFFT_EM) sp->kind = K_EM;
  else if (opt->scheme == SCFFT_ACC_EM) sp->kind = K_ACC_EM;
  else sp->kind = K_ACC_MS;
  sp->s0 = sc.sigma0;
  if (!acc && opt->sigma0_set) sp->s0 = cd(opt->sigma0.re, opt->sigma0.im);
  if (std::abs(sp->s0) == 0.0) return SCFFT_ERR_INVALID_ARG;
  return SCFFT_OK;
}

// Reference conductivity of a graded medium from its extreme conductivities
// (the device computes the extremes; sigma is 1 + (sigma1-1) rho, rho in [0,1]).
cd graded_sigma0(int scheme, cd s1) {
  // sigma ranges over the segment [1, sigma1]
  if (scheme == SCFFT_MS) return (s1 + 1.0) / 2.0;
  return std::sqrt(s1);
}

// Real-field mode: every coefficient real, an x length with a real-field x
// pass and an even number of x lines (rows are transformed in pairs).  Power
// of two: always.  Compile-time mixed-radix lengths: in 3D, and in 2D at
// fp64 (measured, one accelerated iteration: 240^3 fp32 1.57 -> 0.88 ms,
// fp64 4.08 -> 2.26 ms, 480^3 fp32 13.0 -> 7.2 ms, 960^2 fp64 125 -> 90 us;
// but 720^2 and 960^2 fp32 60 -> 64 and 68 -> 77 us: half as many rows and
// columns leave a single 2D solve's passes with too few workgroups).
bool real_ok(const SolveSpec& sp, int d, const int* n, int prec) {
  if (std::getenv("SCFFT_NO_REAL")) return false;
  const bool sm_x = !std::getenv("SCFFT_NO_SMOOTH") && smooth_lines(n[0], 8) > 0 &&
                    (d == 3 || prec == SCFFT_FP64);
  if (!is_p2(n[0]) && !sm_x) return false;
  const long long lines = (long long)n[1] * (d == 3 ? n[2] : 1);
  if (lines % 2) return false;
  if (sp.s1.imag() != 0.0 || sp.s0.imag() != 0.0) return false;
  if (sp.kind == K_ACC_EM || sp.kind == K_ACC_MS) {
    if (sp.sc.t.imag() != 0.0 || !(sp.sc.t.real() > 0.0)) return false;
    if (sp.sc.p[0].imag() != 0.0 || sp.sc.p[1].real() != 0.0 || sp.sc.p[2].real() != 0.0)
      return false;
  }
  return true;
}

}  // namespace
}  // namespace scfft

using namespace scfft;

extern "C" {

void scfft_default_options(scfft_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->scheme = SCFFT_ACC_EM;
  o->precision = SCFFT_FP64;
  o->symbol = SCFFT_GAMMA_ROTATED;
  o->alpha = 0.25;
  o->beta = 4.0;
  o->tol = 1e-8;
  o->max_iter = 1000;
  o->check_every = 16;
  o->stag_window = 20;
  o->div_factor = 1e3;
  o->stream = nullptr;
}

const char* scfft_status_string(int s) {
  switch (s) {
    case SCFFT_OK: return "ok";
    case SCFFT_ERR_INVALID_ARG: return "invalid argument";
    case SCFFT_ERR_SLIT: return "sigma1 lies on the scheme's slit";
    case SCFFT_ERR_NOT_CONVERGED: return "not converged within max_iter";
    case SCFFT_ERR_DIVERGED: return "diverged";
    case SCFFT_ERR_STAGNATED: return "stagnated";
    case SCFFT_ERR_DEVICE: return "HIP device error";
    case SCFFT_ERR_OOM: return "out of device memory";
    default: return "unknown status";
  }
}

const char* scfft_version(void) { return "scfft 0.1 (gfx950)"; }

void scfft_release(void) {
  std::lock_guard<std::mutex> lk(g_mutex);
  free_graphs();
  for (auto& kv : g_plans) free_plan(kv.second);
  g_plans.clear();
}

scfft_status scfft_scheme_scalars(int scheme, scfft_c64 sigma1, double alpha, double beta,
                                  scfft_c64* out) {
  if (!out) return SCFFT_ERR_INVALID_ARG;
  Scalars sc{};
  scfft_status rc = scheme_scalars(scheme, cd(sigma1.re, sigma1.im), alpha, beta, &sc);
  if (rc != SCFFT_OK) return rc;
  const cd v[8] = {sc.sigma0, sc.t, sc.z, sc.p[0], sc.p[1], sc.p[2], sc.e2p, sc.j3p};
  for (int i = 0; i < 8; ++i) {
    out[i].re = v[i].real();
    out[i].im = v[i].imag();
  }
  return SCFFT_OK;
}

scfft_c64 scfft_sigma1_from_z(double a, double b, scfft_c64 zz) {
  const cd z(zz.re, zz.im);
  const cd w = (1.0 + z) / (1.0 - z);
  const cd t = w * w;
  // t (s + b)(1 + a) = (s + a)(1 + b), solved for s
  const cd s = (a * (1.0 + b) - t * b * (1.0 + a)) / (t * (1.0 + a) - (1.0 + b));
  return scfft_c64{s.real(), s.imag()};
}

scfft_status scfft_solve(const scfft_problem* prob, const scfft_options* opt, scfft_result* res) {
  if (!res) return SCFFT_ERR_INVALID_ARG;
  SolveSpec sp{};
  if (!prob) return SCFFT_ERR_INVALID_ARG;
  scfft_status rc = prepare(prob, opt, cd(prob->sigma1.re, prob->sigma1.im), &sp);
  if (rc != SCFFT_OK) {
    res->status = rc;
    return rc;
  }
  if (prob->density && !opt->sigma0_set) sp.s0 = graded_sigma0(opt->scheme, sp.s1);
  std::lock_guard<std::mutex> lk(g_mutex);
  hipStream_t st = reinterpret_cast<hipStream_t>(opt->stream);
  Plan* p = nullptr;
  const bool acc = sp.kind == K_ACC_EM || sp.kind == K_ACC_MS;
  SolveCtl c;
  SolveCoef cf;
  fill_ctl(c, *opt, sp.kind, prob->d, prob->e0);
  fill_coef(cf, sp, prob->density != nullptr, prob->d, prob->e0, (double)voxels(prob));
  const TuneCtx tc{map_kind(sp.kind, prob->density != nullptr), &c, &cf, prob->phase,
                   prob->density};
  rc = get_plan(prob->d, prob->n, opt->precision, 1, acc, opt->symbol, st, &p, 0,
                real_ok(sp, prob->d, prob->n, opt->precision), &tc);
  if (rc != SCFFT_OK) return rc;
  rc = ensure_hist(p, opt->max_iter + 1);
  if (rc != SCFFT_OK) return rc;
  p->mk = tc.mk;
  SCFFT_HIP(hipMemcpyAsync(p->ctl, &c, sizeof(c), hipMemcpyHostToDevice, st));
  SCFFT_HIP(hipMemcpyAsync(p->coef, &cf, sizeof(cf), hipMemcpyHostToDevice, st));
  rc = launch_init(p, st);
  if (rc != SCFFT_OK) return rc;
  double ms = 0;
  std::vector<std::vector<SolveCtl>> fin;
  rc = run_loop({p}, {prob->phase}, {prob->density}, opt->max_iter, opt->check_every, st, &ms,
                true, nullptr, &fin);
  if (rc != SCFFT_OK) return rc;
  return read_result(p, 0, prob, res, st, ms, &fin[0][0]);
}

scfft_status scfft_plan_info(const scfft_problem* prob, const scfft_options* opt, int* info,
                             int cap) {
  if (!prob || !opt || !info || cap < 10) return SCFFT_ERR_INVALID_ARG;
  SolveSpec sp{};
  scfft_status rc = prepare(prob, opt, cd(prob->sigma1.re, prob->sigma1.im), &sp);
  if (rc != SCFFT_OK) return rc;
  if (prob->density && !opt->sigma0_set) sp.s0 = graded_sigma0(opt->scheme, sp.s1);
  std::lock_guard<std::mutex> lk(g_mutex);
  hipStream_t st = reinterpret_cast<hipStream_t>(opt->stream);
  Plan* p = nullptr;
  const bool acc = sp.kind == K_ACC_EM || sp.kind == K_ACC_MS;
  SolveCtl c;
  SolveCoef cf;
  fill_ctl(c, *opt, sp.kind, prob->d, prob->e0);
  fill_coef(cf, sp, prob->density != nullptr, prob->d, prob->e0, (double)voxels(prob));
  const TuneCtx tc{map_kind(sp.kind, prob->density != nullptr), &c, &cf, prob->phase,
                   prob->density};
  rc = get_plan(prob->d, prob->n, opt->precision, 1, acc, opt->symbol, st, &p, 0,
                real_ok(sp, prob->d, prob->n, opt->precision), &tc);
  if (rc != SCFFT_OK) return rc;
  const int v[13] = {p->real ? 1 : 0, p->packed ? 1 : 0, p->kn.pitch, p->kn.nt, p->kn.xr,
                     p->kn.gr, p->gC, p->d == 3 ? p->yC : 0, p->tuned ? 1 : 0, p->xL,
                     p->p2x ? 1 : p->smx ? 2 : 0, p->p2g ? 1 : p->smg ? 2 : 0,
                     p->d != 3 ? 0 : p->p2y ? 1 : p->smy ? 2 : 0};
  for (int i = 0; i < std::min(cap, 13); ++i) info[i] = v[i];
  return SCFFT_OK;
}

scfft_status scfft_effective_tensor(const scfft_problem* prob, const scfft_options* opt,
                                    scfft_c64* tensor, int* iterations) {
  if (!prob || !opt || !tensor) return SCFFT_ERR_INVALID_ARG;
  scfft_problem pr = *prob;
  for (int i = 0; i < 3; ++i) pr.e0[i] = i == 0 ? 1.0 : 0.0;
  SolveSpec sp{};
  scfft_status rc = prepare(&pr, opt, cd(prob->sigma1.re, prob->sigma1.im), &sp);
  if (rc != SCFFT_OK) return rc;
  if (prob->density && !opt->sigma0_set) sp.s0 = graded_sigma0(opt->scheme, sp.s1);
  std::lock_guard<std::mutex> lk(g_mutex);
  hipStream_t st = reinterpret_cast<hipStream_t>(opt->stream);
  const int d = prob->d;
  Plan* p = nullptr;
  const bool acc = sp.kind == K_ACC_EM || sp.kind == K_ACC_MS;
  std::vector<SolveCtl> c(d);
  std::vector<SolveCoef> cf(d);
  for (int j = 0; j < d; ++j) {
    double e0[3] = {0.0, 0.0, 0.0};
    e0[j] = 1.0;
    fill_ctl(c[j], *opt, sp.kind, d, e0);
    fill_coef(cf[j], sp, prob->density != nullptr, d, e0, (double)voxels(prob));
  }
  const TuneCtx tc{map_kind(sp.kind, prob->density != nullptr), &c[0], &cf[0], prob->phase,
                   prob->density};
  rc = get_plan(d, prob->n, opt->precision, d, acc, opt->symbol, st, &p, 0,
                real_ok(sp, d, prob->n, opt->precision), &tc);
  if (rc != SCFFT_OK) return rc;
  rc = ensure_hist(p, opt->max_iter + 1);
  if (rc != SCFFT_OK) return rc;
  p->mk = map_kind(sp.kind, prob->density != nullptr);
  SCFFT_HIP(hipMemcpyAsync(p->ctl, c.data(), sizeof(SolveCtl) * d, hipMemcpyHostToDevice, st));
  SCFFT_HIP(hipMemcpyAsync(p->coef, cf.data(), sizeof(SolveCoef) * d, hipMemcpyHostToDevice, st));
  rc = launch_init(p, st);
  if (rc != SCFFT_OK) return rc;
  double ms = 0;
  rc = run_loop({p}, {prob->phase}, {prob->density}, opt->max_iter, opt->check_every, st, &ms);
  if (rc != SCFFT_OK) return rc;
  SCFFT_HIP(hipMemcpyAsync(c.data(), p->ctl, sizeof(SolveCtl) * d, hipMemcpyDeviceToHost, st));
  SCFFT_HIP(hipStreamSynchronize(st));
  scfft_status worst = SCFFT_OK;
  for (int j = 0; j < d; ++j) {
    for (int i = 0; i < d; ++i) {
      tensor[i * d + j].re = c[j].meanJ[2 * i];
      tensor[i * d + j].im = c[j].meanJ[2 * i + 1];
    }
    if (iterations) iterations[j] = c[j].iter;
    if (c[j].status < worst) worst = (scfft_status)c[j].status;
  }
  return worst;
}

scfft_status scfft_series_coefficients(const scfft_problem* prob, const scfft_options* opt,
                                       int nterms, scfft_c64* coeffs) {
  if (!prob || !opt || !coeffs || nterms < 1 || nterms > 100000) return SCFFT_ERR_INVALID_ARG;
  if (!prob->phase || prob->density) return SCFFT_ERR_INVALID_ARG;
  scfft_options o = *opt;
  o.scheme = SCFFT_ACC_EM;
  o.tol = -1.0;
  o.max_iter = nterms;
  o.stag_window = 0;
  o.div_factor = 0.0;
  SolveSpec sp{};
  // sigma1 = 1 gives t = 1; only p (from alpha, beta) enters the operator K
  scfft_status rc = prepare(prob, &o, cd(1.0, 0.0), &sp);
  if (rc != SCFFT_OK) return rc;
  std::lock_guard<std::mutex> lk(g_mutex);
  hipStream_t st = reinterpret_cast<hipStream_t>(o.stream);
  Plan* p = nullptr;
  SolveCtl c;
  SolveCoef cf;
  fill_ctl(c, o, sp.kind, prob->d, prob->e0);
  fill_coef(cf, sp, false, prob->d, prob->e0, (double)voxels(prob));
  // z = 1 and no source: the local map returns K x, and with s1 = 1,
  // inv1w = -1, p1kap = 2 p1 its "physical field" E = -x + 2 p1 s (phase 1),
  // -x (phase 2) is (K x)_Q, so the reduced <J> = <E> is <(K u)_Q>
  put(cf.s1, cd(1.0, 0.0));
  put(cf.z, cd(1.0, 0.0));
  put(cf.inv1w, cd(-1.0, 0.0));
  put(cf.p1kap, 2.0 * sp.sc.p[0]);
  for (int i = 0; i < prob->d; ++i) {
    put(cf.kz_src[i], cd(0.0, 0.0));
    put(cf.init_src[i], cd((double)voxels(prob) * prob->e0[i], 0.0));
  }
  const TuneCtx tc{map_kind(sp.kind, false), &c, &cf, prob->phase, nullptr};
  rc = get_plan(prob->d, prob->n, o.precision, 1, true, o.symbol, st, &p, 0,
                real_ok(sp, prob->d, prob->n, o.precision), &tc);
  if (rc != SCFFT_OK) return rc;
  rc = ensure_hist(p, nterms + 1);
  if (rc != SCFFT_OK) return rc;
  p->mk = tc.mk;
  SCFFT_HIP(hipMemcpyAsync(p->ctl, &c, sizeof(c), hipMemcpyHostToDevice, st));
  SCFFT_HIP(hipMemcpyAsync(p->coef, &cf, sizeof(cf), hipMemcpyHostToDevice, st));
  rc = launch_init(p, st);
  if (rc != SCFFT_OK) return rc;
  double ms = 0;
  rc = run_loop({p}, {prob->phase}, {nullptr}, nterms, o.check_every, st, &ms);
  if (rc != SCFFT_OK) return rc;
  std::vector<double> hs(2 * (size_t)nterms);
  SCFFT_HIP(hipMemcpyAsync(hs.data(), p->hist_s, sizeof(double) * hs.size(), hipMemcpyDeviceToHost, st));
  SCFFT_HIP(hipMemcpyAsync(&c, p->ctl, sizeof(c), hipMemcpyDeviceToHost, st));
  SCFFT_HIP(hipStreamSynchronize(st));
  // iteration n reduces <(K u_n)_Q>; a non-finite stop leaves later entries unset
  const int valid = c.status == SCFFT_ERR_DIVERGED ? std::min(c.iter, nterms) : nterms;
  coeffs[0] = scfft_c64{1.0, 0.0};
  for (int k = 1; k <= nterms; ++k) {
    if (k - 1 < valid) {
      coeffs[k] = scfft_c64{2.0 * hs[2 * (k - 1)], 2.0 * hs[2 * (k - 1) + 1]};
    } else {
      coeffs[k] = scfft_c64{NAN, NAN};
    }
  }
  return SCFFT_OK;
}

scfft_status scfft_series_evaluate(int nterms, const scfft_c64* coeffs, double alpha, double beta,
                                   int pade_m, int nsig, const scfft_c64* sigma1s,
                                   scfft_c64* out) {
  if (nterms < 0 || nterms > 100000 || !coeffs || nsig < 0 || pade_m < 0 || pade_m > nterms)
    return SCFFT_ERR_INVALID_ARG;
  if (nsig > 0 && (!sigma1s || !out)) return SCFFT_ERR_INVALID_ARG;
  if (!(alpha > 0.0) || !(beta > alpha) || !std::isfinite(beta)) return SCFFT_ERR_INVALID_ARG;
  std::vector<cd> c(nterms + 1);
  for (int k = 0; k <= nterms; ++k) c[k] = cd(coeffs[k].re, coeffs[k].im);
  auto cc = [&](int i) { return (i >= 0 && i <= nterms) ? c[i] : cd(0.0, 0.0); };
  const int M = pade_m, L = nterms - pade_m;
  std::vector<cd> q(M + 1, cd(0.0, 0.0)), a(L + 1, cd(0.0, 0.0));
  q[0] = 1.0;
  if (M > 0) {
    // sum_{j=1..M} q_j c_{L+i-j} = -c_{L+i}, i = 1..M: LU with partial pivoting
    std::vector<cd> A((size_t)M * M), b(M);
    for (int i = 0; i < M; ++i) {
      for (int j = 0; j < M; ++j) A[(size_t)i * M + j] = cc(L + (i + 1) - (j + 1));
      b[i] = -cc(L + i + 1);
    }
    for (int k = 0; k < M; ++k) {
      int piv = k;
      for (int i = k + 1; i < M; ++i)
        if (std::abs(A[(size_t)i * M + k]) > std::abs(A[(size_t)piv * M + k])) piv = i;
      if (!(std::abs(A[(size_t)piv * M + k]) > 0.0)) return SCFFT_ERR_INVALID_ARG;
      if (piv != k) {
        for (int j = 0; j < M; ++j) std::swap(A[(size_t)k * M + j], A[(size_t)piv * M + j]);
        std::swap(b[k], b[piv]);
      }
      for (int i = k + 1; i < M; ++i) {
        const cd f = A[(size_t)i * M + k] / A[(size_t)k * M + k];
        for (int j = k; j < M; ++j) A[(size_t)i * M + j] -= f * A[(size_t)k * M + j];
        b[i] -= f * b[k];
      }
    }
    for (int k = M - 1; k >= 0; --k) {
      cd v = b[k];
      for (int j = k + 1; j < M; ++j) v -= A[(size_t)k * M + j] * q[j + 1];
      q[k + 1] = v / A[(size_t)k * M + k];
    }
  }
  for (int i = 0; i <= L; ++i) {
    cd v(0.0, 0.0);
    for (int j = 0; j <= std::min(i, M); ++j) v += q[j] * c[i - j];
    a[i] = v;
  }
  for (int n = 0; n < nsig; ++n) {
    const cd s(sigma1s[n].re, sigma1s[n].im);
    if (s.imag() == 0.0 && s.real() >= -beta && s.real() <= -alpha) return SCFFT_ERR_SLIT;
    const cd t = (s + alpha) * (1.0 + beta) / ((s + beta) * (1.0 + alpha));   // eq. J6
    const cd w = std::sqrt(t);
    const cd z = (w - 1.0) / (w + 1.0);                                      // eq. J7
    cd num(0.0, 0.0), den(0.0, 0.0);
    for (int i = L; i >= 0; --i) num = num * z + a[i];
    for (int j = M; j >= 0; --j) den = den * z + q[j];
    const cd v = w * num / den;
    out[n] = scfft_c64{v.real(), v.imag()};
  }
  return SCFFT_OK;
}

scfft_status scfft_solve_batch(int nprob, const scfft_problem* probs, const scfft_options* opts,
                               int nsig, const scfft_c64* sigma1s, scfft_result* results) {
  if (nprob <= 0 || nsig <= 0 || nsig > 256 || !probs || !opts || !sigma1s || !results)
    return SCFFT_ERR_INVALID_ARG;
  const scfft_options& o0 = opts[0];
  std::vector<std::vector<SolveSpec>> specs(nprob, std::vector<SolveSpec>(nsig));
  bool any_acc = false;
  for (int i = 0; i < nprob; ++i)
    for (int j = 0; j < nsig; ++j) {
      scfft_options o = opts[i];
      o.precision = o0.precision;
      o.symbol = o0.symbol;
      const scfft_c64 s = sigma1s[(size_t)i * nsig + j];
      scfft_status rc = prepare(&probs[i], &o, cd(s.re, s.im), &specs[i][j]);
      if (rc != SCFFT_OK) {
        results[(size_t)i * nsig + j].status = rc;
        return rc;
      }
      if (probs[i].density && !o.sigma0_set) specs[i][j].s0 = graded_sigma0(o.scheme, specs[i][j].s1);
      any_acc |= specs[i][j].kind == K_ACC_EM || specs[i][j].kind == K_ACC_MS;
    }
  std::lock_guard<std::mutex> lk(g_mutex);
  hipStream_t st = reinterpret_cast<hipStream_t>(o0.stream);
  std::vector<Plan*> plans(nprob);
  std::vector<const uint8_t*> ph(nprob);
  std::vector<const double*> de(nprob);
  for (int i = 0; i < nprob; ++i) {
    bool real = true;
    for (int j = 0; j < nsig; ++j)
      real = real && real_ok(specs[i][j], probs[i].d, probs[i].n, o0.precision);
    std::vector<SolveCtl> c(nsig);
    std::vector<SolveCoef> cf(nsig);
    for (int j = 0; j < nsig; ++j) {
      fill_ctl(c[j], o0, specs[i][j].kind, probs[i].d, probs[i].e0);
      fill_coef(cf[j], specs[i][j], probs[i].density != nullptr, probs[i].d, probs[i].e0,
                (double)voxels(&probs[i]));
    }
    // knobs tuned on one solve of this structure
    const TuneCtx tc{map_kind(specs[i][0].kind, probs[i].density != nullptr), &c[0], &cf[0],
                     probs[i].phase, probs[i].density};
    scfft_status rc = get_plan(probs[i].d, probs[i].n, o0.precision, nsig, any_acc, o0.symbol, st,
                               &plans[i], i, real, &tc);
    if (rc != SCFFT_OK) return rc;
    rc = ensure_hist(plans[i], o0.max_iter + 1);
    if (rc != SCFFT_OK) return rc;
    plans[i]->mk = tc.mk;
    for (int j = 1; j < nsig; ++j)
      if (map_kind(specs[i][j].kind, probs[i].density != nullptr) != plans[i]->mk)
        return SCFFT_ERR_INVALID_ARG;
    SCFFT_HIP(hipMemcpyAsync(plans[i]->ctl, c.data(), sizeof(SolveCtl) * nsig,
                             hipMemcpyHostToDevice, st));
    SCFFT_HIP(hipMemcpyAsync(plans[i]->coef, cf.data(), sizeof(SolveCoef) * nsig,
                             hipMemcpyHostToDevice, st));
    SCFFT_HIP(hipStreamSynchronize(st));
    rc = launch_init(plans[i], st);
    if (rc != SCFFT_OK) return rc;
    ph[i] = probs[i].phase;
    de[i] = probs[i].density;
  }
  double ms = 0;
  std::vector<std::vector<SolveCtl>> fin;
  scfft_status rc = run_loop(plans, ph, de, o0.max_iter, o0.check_every, st, &ms, true, nullptr,
                             &fin);
  if (rc != SCFFT_OK) return rc;
  scfft_status worst = SCFFT_OK;
  for (int i = 0; i < nprob; ++i)
    for (int j = 0; j < nsig; ++j) {
      scfft_result* r = &results[(size_t)i * nsig + j];
      scfft_status s = read_result(plans[i], j, &probs[i], r, st, ms, &fin[i][j]);
      if (s == SCFFT_ERR_DEVICE || s == SCFFT_ERR_OOM) return s;
      if (s < worst) worst = s;
    }
  return worst;
}

scfft_status scfft_estimate_interval(const scfft_problem* prob, int iters, int symbol,
                                     void* stream, double* alpha, double* beta, double* mu_min,
                                     double* mu_max) {
  if (!prob || !prob->phase || iters < 0 || symbol < 0 || symbol > 2) return SCFFT_ERR_INVALID_ARG;
  scfft_status rc = check_dims(prob->d, prob->n, SCFFT_FP64);
  if (rc != SCFFT_OK) return rc;
  std::lock_guard<std::mutex> lk(g_mutex);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  Plan* p = nullptr;
  SolveSpec pw{};
  pw.kind = K_POWER;
  scfft_options o;
  scfft_default_options(&o);
  o.tol = -1.0;
  o.max_iter = iters + 1;
  o.stag_window = 0;
  o.div_factor = 0.0;
  const double e0[3] = {1.0, 0.0, 0.0};
  SolveCtl c[2];
  SolveCoef cf[2];
  for (int k = 0; k < 2; ++k) {
    SolveSpec sp{};
    sp.kind = K_POWER;
    sp.power_phase = k == 0 ? 1 : 0;
    fill_ctl(c[k], o, K_POWER, prob->d, e0);
    fill_coef(cf[k], sp, false, prob->d, e0, (double)voxels(prob));
  }
  const TuneCtx tc{MAP_LIN, &c[0], &cf[0], prob->phase, nullptr};
  rc = get_plan(prob->d, prob->n, SCFFT_FP64, 2, false, symbol, st, &p, 0,
                real_ok(pw, prob->d, prob->n, SCFFT_FP64), &tc);
  if (rc != SCFFT_OK) return rc;
  rc = ensure_hist(p, iters + 2);
  if (rc != SCFFT_OK) return rc;
  p->mk = MAP_LIN;
  SCFFT_HIP(hipMemcpyAsync(p->ctl, c, sizeof(c), hipMemcpyHostToDevice, st));
  SCFFT_HIP(hipMemcpyAsync(p->coef, cf, sizeof(cf), hipMemcpyHostToDevice, st));
  rc = launch_init(p, st);
  if (rc != SCFFT_OK) return rc;
  double ms = 0;
  rc = run_loop({p}, {prob->phase}, {nullptr}, o.max_iter, 32, st, &ms);
  if (rc != SCFFT_OK) return rc;
  SolveCtl h[2];
  SCFFT_HIP(hipMemcpyAsync(h, p->ctl, sizeof(h), hipMemcpyDeviceToHost, st));
  SCFFT_HIP(hipStreamSynchronize(st));
  const double mmax = h[0].lam;
  const double mmin = 1.0 - h[1].lam;
  if (mu_max) *mu_max = mmax;
  if (mu_min) *mu_min = mmin;
  if (alpha) *alpha = 1.0 / mmax - 1.0;
  if (beta) *beta = 1.0 / mmin - 1.0;
  return SCFFT_OK;
}

// Lanczos process on A = Gamma_1 chi Gamma_1 from v_0 = Gamma_1 chi e0 (fp64)
// with full reorthogonalisation: q_0 = v_0/|v_0|; step j applies A to q_j
// (one x pass and one Gamma pass, the power-iteration map with weight chi),
// removes the components along q_0..q_j by classical Gram-Schmidt twice
// (a_j = the total removed along q_j), and b_{j+1} = |r|, q_{j+1} = r/b_{j+1}.
// All vectors stay in the passes' stored spectral form (kernels_lanczos.hpp);
// the basis lives in a buffer of (steps + 1) vectors allocated for the call.
// The process stops after `steps` values of a, or when
// b_{j+1} < 1e-12 max(1, |a_j|) (the Krylov space closed).
scfft_status lanczos_run(const scfft_problem* prob, int steps, int symbol, hipStream_t st,
                         std::vector<double>& a, std::vector<double>& b, double* norm0,
                         double* b_last = nullptr) {
  if (!prob || !prob->phase || prob->density || steps < 1 || steps > 200 || symbol < 0 ||
      symbol > 2 || bad_e0(prob))
    return SCFFT_ERR_INVALID_ARG;
  scfft_status rc = check_dims(prob->d, prob->n, SCFFT_FP64);
  if (rc != SCFFT_OK) return rc;
  std::lock_guard<std::mutex> lk(g_mutex);
  Plan* p = nullptr;
  SolveSpec pw{};
  pw.kind = K_POWER;
  pw.power_phase = 1;
  scfft_options o;
  scfft_default_options(&o);
  o.tol = -1.0;
  o.max_iter = steps + 1;
  o.stag_window = 0;
  o.div_factor = 0.0;
  SolveCtl c;
  SolveCoef cf;
  fill_ctl(c, o, K_POWER, prob->d, prob->e0);
  fill_coef(cf, pw, false, prob->d, prob->e0, (double)voxels(prob));
  const TuneCtx tc{MAP_LIN, &c, &cf, prob->phase, nullptr};
  rc = get_plan(prob->d, prob->n, SCFFT_FP64, 1, false, symbol, st, &p, 0,
                real_ok(pw, prob->d, prob->n, SCFFT_FP64), &tc);
  if (rc != SCFFT_OK) return rc;
  p->mk = MAP_LIN;
  SCFFT_HIP(hipMemcpyAsync(p->ctl, &c, sizeof(c), hipMemcpyHostToDevice, st));
  SCFFT_HIP(hipMemcpyAsync(p->coef, &cf, sizeof(cf), hipMemcpyHostToDevice, st));
  rc = launch_init(p, st);
  if (rc != SCFFT_OK) return rc;

  LzArgs z{};
  z.X = reinterpret_cast<cx<double>*>(p->X);
  z.vlen = (long long)p->d * p->Mh;
  z.H = p->H;
  z.HP = p->HP;
  z.half = p->real ? 1 : 0;
  z.packed = p->packed ? 1 : 0;
  const int nb = (int)std::min<long long>((z.vlen + kLzThreads - 1) / kLzThreads, 1024);
  const size_t vbytes = sizeof(cx<double>) * (size_t)z.vlen;
  void* qbuf = nullptr;
  double* work = nullptr;   // part [201][nb][2], red [201][2], per-step scalars [steps+1][3]
  const size_t nwork = (size_t)201 * nb * 2 + 201 * 2 + (size_t)(steps + 1) * 3;
  if (hipMalloc(&qbuf, vbytes * (size_t)(steps + 1)) != hipSuccess) return SCFFT_ERR_OOM;
  if (hipMalloc(&work, sizeof(double) * nwork) != hipSuccess) {
    (void)hipFree(qbuf);
    return SCFFT_ERR_OOM;
  }
  z.Q = static_cast<cx<double>*>(qbuf);
  z.part = work;
  z.red = work + (size_t)201 * nb * 2;
  double* scal = z.red + 201 * 2;
  const double nd = (double)p->M;
  auto dots_and_update = [&](int nk, double* save) {
    z.nk = nk;
    z.save = save;
    z.save_k = nk - 1;
    const dim3 g((unsigned)nb, (unsigned)((nk + kLzGroup - 1) / kLzGroup));
    hipLaunchKernelGGL(lz_dots_kernel, g, dim3(kLzThreads), 0, st, z);
    hipLaunchKernelGGL(lz_reduce_kernel, dim3(nk), dim3(kLzThreads), 0, st, z, nb);
    hipLaunchKernelGGL(lz_update_kernel, dim3(nb), dim3(kLzThreads), 0, st, z);
  };
  auto norm = [&](double* save) {
    z.nk = 1;
    z.save = save;
    z.save_k = 0;
    hipLaunchKernelGGL(lz_norm_kernel, dim3(nb), dim3(kLzThreads), 0, st, z);
    hipLaunchKernelGGL(lz_reduce_kernel, dim3(1), dim3(kLzThreads), 0, st, z, nb);
  };
  auto scale_into = [&](int slot) {
    z.slot = slot;
    hipLaunchKernelGGL(lz_scale_kernel, dim3(nb), dim3(kLzThreads), 0, st, z);
  };
  a.clear();
  b.clear();
  do {
    // v_0 = Gamma_1 chi e0 (the power map applied to the source e0)
    rc = launch_iteration(p, prob->phase, nullptr, st, true);
    if (rc != SCFFT_OK) break;
    norm(scal);
    double h[3] = {0, 0, 0};
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(h, scal, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      rc = SCFFT_ERR_DEVICE;
      break;
    }
    // Parseval: X holds the x-spectrum of the field times N^d/n0
    const double n0 = h[0] * (double)p->n[0] / (nd * nd);
    if (!(n0 > 0.0) || !std::isfinite(n0)) {
      rc = SCFFT_ERR_INVALID_ARG;   // v_0 = 0: e0 sees no inhomogeneity
      break;
    }
    if (norm0) *norm0 = n0;
    scale_into(0);
    for (int j = 0; j < steps; ++j) {
      rc = launch_iteration(p, prob->phase, nullptr, st, true);   // X = A q_j
      if (rc != SCFFT_OK) break;
      double* sj = scal + 3 * (size_t)j;
      dots_and_update(j + 1, sj);       // classical Gram-Schmidt ...
      dots_and_update(j + 1, sj + 1);   // ... twice
      norm(sj + 2);
      if (hipGetLastError() != hipSuccess ||
          hipMemcpyAsync(h, sj, 3 * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess) {
        rc = SCFFT_ERR_DEVICE;
        break;
      }
      const double aj = h[0] + h[1], bj = std::sqrt(std::max(h[2], 0.0));
      if (!std::isfinite(aj) || !std::isfinite(bj)) {
        rc = SCFFT_ERR_DEVICE;
        break;
      }
      a.push_back(aj);
      if (j == steps - 1 || bj < 1e-12 * std::max(1.0, std::fabs(aj))) {
        if (b_last) *b_last = j == steps - 1 ? bj : 0.0;
        break;
      }
      b.push_back(bj);
      scale_into(j + 1);
    }
  } while (false);
  (void)hipStreamSynchronize(st);
  (void)hipFree(qbuf);
  (void)hipFree(work);
  if (rc != SCFFT_OK) return rc;
  if (a.empty()) return SCFFT_ERR_INVALID_ARG;
  return SCFFT_OK;
}

// Gauss rule of the symmetric tridiagonal matrix (a, b): eigenvalues and
// squared first eigenvector components (cyclic Jacobi rotations on the
// dense matrix; m <= 200).
void gauss_rule(const std::vector<double>& a, const std::vector<double>& b, std::vector<double>& node,
                std::vector<double>& w0) {
  const int m = (int)a.size();
  std::vector<double> A((size_t)m * m, 0.0), V((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i) {
    A[(size_t)i * m + i] = a[i];
    V[(size_t)i * m + i] = 1.0;
    if (i + 1 < m) A[(size_t)i * m + i + 1] = A[(size_t)(i + 1) * m + i] = b[i];
  }
  double scale = 0;
  for (double v : A) scale += v * v;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0;
    for (int i = 0; i < m; ++i)
      for (int j = i + 1; j < m; ++j) off += A[(size_t)i * m + j] * A[(size_t)i * m + j];
    if (off <= 1e-32 * scale) break;
    for (int pp = 0; pp < m; ++pp)
      for (int q = pp + 1; q < m; ++q) {
        const double apq = A[(size_t)pp * m + q];
        if (apq == 0.0) continue;
        const double th = (A[(size_t)q * m + q] - A[(size_t)pp * m + pp]) / (2.0 * apq);
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
        for (int k = 0; k < m; ++k) {   // columns pp, q
          const double akp = A[(size_t)k * m + pp], akq = A[(size_t)k * m + q];
          A[(size_t)k * m + pp] = cs * akp - sn * akq;
          A[(size_t)k * m + q] = sn * akp + cs * akq;
        }
        for (int k = 0; k < m; ++k) {   // rows pp, q
          const double apk = A[(size_t)pp * m + k], aqk = A[(size_t)q * m + k];
          A[(size_t)pp * m + k] = cs * apk - sn * aqk;
          A[(size_t)q * m + k] = sn * apk + cs * aqk;
        }
        for (int k = 0; k < m; ++k) {
          const double vkp = V[(size_t)k * m + pp], vkq = V[(size_t)k * m + q];
          V[(size_t)k * m + pp] = cs * vkp - sn * vkq;
          V[(size_t)k * m + q] = sn * vkp + cs * vkq;
        }
      }
  }
  node.resize(m);
  w0.resize(m);
  for (int i = 0; i < m; ++i) {
    node[i] = A[(size_t)i * m + i];
    w0[i] = V[i] * V[i];   // first row of V: first components of the eigenvectors
  }
}

scfft_status scfft_lanczos(const scfft_problem* prob, int steps, int symbol, void* stream,
                           double* a, double* b, double* norm0, int* m) {
  if (!a || !b || !m) return SCFFT_ERR_INVALID_ARG;
  std::vector<double> va, vb;
  double bl = 0.0;
  scfft_status rc = lanczos_run(prob, steps, symbol, reinterpret_cast<hipStream_t>(stream), va, vb,
                                norm0, &bl);
  if (rc != SCFFT_OK) return rc;
  *m = (int)va.size();
  for (size_t i = 0; i < va.size(); ++i) a[i] = va[i];
  for (size_t i = 0; i < vb.size(); ++i) b[i] = vb[i];
  b[va.size() - 1] = bl;
  return SCFFT_OK;
}

scfft_status scfft_estimate_interval_lanczos(const scfft_problem* prob, int steps, int symbol,
                                             void* stream, double rel_weight, double* alpha,
                                             double* beta, double* alpha_used, double* beta_used,
                                             double* mu_min, double* mu_max) {
  if (!(rel_weight >= 0.0) || !(rel_weight < 1.0)) return SCFFT_ERR_INVALID_ARG;
  std::vector<double> va, vb, node, w0;
  scfft_status rc = lanczos_run(prob, steps, symbol, reinterpret_cast<hipStream_t>(stream), va, vb,
                                nullptr);
  if (rc != SCFFT_OK) return rc;
  gauss_rule(va, vb, node, w0);
  double tot = 0;
  for (double w : w0) tot += w;
  double lo = INFINITY, hi = -INFINITY;
  for (size_t i = 0; i < node.size(); ++i)
    if (w0[i] > rel_weight * tot) {
      lo = std::min(lo, node[i]);
      hi = std::max(hi, node[i]);
    }
  if (!(lo > 0.0) || !(hi < 1.0) || !(lo <= hi)) return SCFFT_ERR_INVALID_ARG;
  const double al = 1.0 / hi - 1.0, be = 1.0 / lo - 1.0;
  // floating-point stability of the accelerated scheme: alpha beta = 1
  const double au = std::min(al, 1.0 / be);
  if (mu_min) *mu_min = lo;
  if (mu_max) *mu_max = hi;
  if (alpha) *alpha = al;
  if (beta) *beta = be;
  if (alpha_used) *alpha_used = au;
  if (beta_used) *beta_used = 1.0 / au;
  return SCFFT_OK;
}

scfft_status scfft_gradient(const scfft_problem* prob, const scfft_options* opt, scfft_c64* g,
                            scfft_c64* drho, scfft_c64* dsigma1, scfft_result* fwd,
                            scfft_result* adj) {
  if (!prob || !opt) return SCFFT_ERR_INVALID_ARG;
  if (opt->symbol == SCFFT_GAMMA_NETWORK) return SCFFT_ERR_INVALID_ARG;
  scfft_options o = *opt;
  o.scheme = SCFFT_EM;
  const cd s1(prob->sigma1.re, prob->sigma1.im);
  SolveSpec sp{};
  scfft_status rc = prepare(prob, &o, s1, &sp);
  if (rc != SCFFT_OK) return rc;
  if (!o.sigma0_set) sp.s0 = std::sqrt(s1);   // sqrt(sigma_min sigma_max) with sigma in [1, sigma1]
  hipStream_t st = reinterpret_cast<hipStream_t>(o.stream);
  double* Ef = nullptr;
  double* part = nullptr;
  double* sum = nullptr;
  const long long M = (long long)prob->n[0] * prob->n[1] * (prob->d == 3 ? prob->n[2] : 1);
  const int gblocks = (int)std::min<long long>((M + 255) / 256, 4096);
  SCFFT_HIP(hipMalloc(&Ef, sizeof(double) * 2 * prob->d * M));
  if (hipMalloc(&part, sizeof(double) * 2 * gblocks) != hipSuccess ||
      hipMalloc(&sum, sizeof(double) * 2) != hipSuccess) {
    (void)hipFree(Ef);
    if (part) (void)hipFree(part);
    return SCFFT_ERR_OOM;
  }
  scfft_result rf{};
  scfft_result ra{};
  if (fwd) rf = *fwd;
  if (adj) ra = *adj;
  rf.E = reinterpret_cast<scfft_c64*>(Ef);
  rf.J = fwd ? fwd->J : nullptr;
  ra.E = nullptr;
  ra.J = nullptr;
  scfft_status out = SCFFT_OK;
  {
    std::lock_guard<std::mutex> lk(g_mutex);
    Plan* p = nullptr;
    SolveCtl c0;
    SolveCoef cf0;
    {
      SolveSpec s = sp;
      s.kind = K_EM;
      fill_ctl(c0, o, s.kind, prob->d, prob->e0);
      fill_coef(cf0, s, prob->density != nullptr, prob->d, prob->e0, (double)M);
    }
    const TuneCtx tc{map_kind(K_EM, prob->density != nullptr), &c0, &cf0, prob->phase,
                     prob->density};
    rc = get_plan(prob->d, prob->n, o.precision, 1, false, o.symbol, st, &p, 0,
                  real_ok(sp, prob->d, prob->n, o.precision), &tc);
    if (rc == SCFFT_OK) rc = ensure_hist(p, o.max_iter + 1);
    for (int pass = 0; pass < 2 && rc == SCFFT_OK; ++pass) {
      SolveSpec s = sp;
      s.kind = pass == 0 ? K_EM : K_ADJ;
      SolveCtl c;
      SolveCoef cf;
      fill_ctl(c, o, s.kind, prob->d, prob->e0);
      fill_coef(cf, s, prob->density != nullptr, prob->d, prob->e0, (double)p->M);
      p->mk = map_kind(s.kind, prob->density != nullptr);
      if (hipMemcpyAsync(p->ctl, &c, sizeof(c), hipMemcpyHostToDevice, st) != hipSuccess ||
          hipMemcpyAsync(p->coef, &cf, sizeof(cf), hipMemcpyHostToDevice, st) != hipSuccess) {
        rc = SCFFT_ERR_DEVICE;
        break;
      }
      rc = launch_init(p, st);
      double ms = 0;
      if (rc == SCFFT_OK)
        rc = run_loop({p}, {prob->phase}, {prob->density}, o.max_iter, o.check_every, st, &ms);
      if (rc != SCFFT_OK) break;
      scfft_status s2 = read_result(p, 0, prob, pass == 0 ? &rf : &ra, st, ms);
      if (s2 == SCFFT_ERR_DEVICE || s2 == SCFFT_ERR_OOM) {
        rc = s2;
        break;
      }
      if (s2 < out) out = s2;
    }
    if (rc == SCFFT_OK) {
      GradArgs a{};
      a.E = Ef;
      a.Y = p->Ep;
      a.phase = prob->phase;
      a.density = prob->density;
      a.g = reinterpret_cast<double*>(g);
      a.drho = reinterpret_cast<double*>(drho);
      a.part = part;
      a.s1[0] = s1.real();
      a.s1[1] = s1.imag();
      a.s0[0] = sp.s0.real();
      a.s0[1] = sp.s0.imag();
      double n2 = 0;
      for (int i = 0; i < prob->d; ++i) {
        a.e0[i] = prob->e0[i];
        n2 += prob->e0[i] * prob->e0[i];
      }
      a.scale = 1.0 / ((double)M * n2);
      a.M = M;
      a.d = prob->d;
      if (o.precision == SCFFT_FP32) {
        if (p->real)
          hipLaunchKernelGGL((gradient_kernel<float, true>), dim3(gblocks), dim3(256), 0, st, a);
        else
          hipLaunchKernelGGL((gradient_kernel<float, false>), dim3(gblocks), dim3(256), 0, st, a);
      } else {
        if (p->real)
          hipLaunchKernelGGL((gradient_kernel<double, true>), dim3(gblocks), dim3(256), 0, st, a);
        else
          hipLaunchKernelGGL((gradient_kernel<double, false>), dim3(gblocks), dim3(256), 0, st, a);
      }
      hipLaunchKernelGGL(sum_pairs_kernel, dim3(1), dim3(256), 0, st, part, gblocks, sum);
      double hs[2] = {0, 0};
      if (hipGetLastError() != hipSuccess ||
          hipMemcpyAsync(hs, sum, sizeof(hs), hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        rc = SCFFT_ERR_DEVICE;
      if (dsigma1) {
        dsigma1->re = hs[0];
        dsigma1->im = hs[1];
      }
    }
  }
  if (fwd) {
    scfft_c64* keepE = fwd->E;
    *fwd = rf;
    fwd->E = keepE;
    if (keepE && rc == SCFFT_OK)
      (void)hipMemcpyAsync(keepE, Ef, sizeof(double) * 2 * prob->d * M, hipMemcpyDeviceToDevice, st);
  }
  if (adj) {
    scfft_c64* kE = adj->E;
    scfft_c64* kJ = adj->J;
    *adj = ra;
    adj->E = kE;
    adj->J = kJ;
  }
  (void)hipStreamSynchronize(st);
  (void)hipFree(Ef);
  (void)hipFree(part);
  (void)hipFree(sum);
  if (rc != SCFFT_OK) return rc;
  return out;
}

scfft_status scfft_profile_passes(const scfft_problem* prob, const scfft_options* opt, int iters,
                                  double* ms, int cap) {
  if (!prob || !opt || !ms || cap < 5 || iters < 1) return SCFFT_ERR_INVALID_ARG;
  SolveSpec sp{};
  scfft_status rc = prepare(prob, opt, cd(prob->sigma1.re, prob->sigma1.im), &sp);
  if (rc != SCFFT_OK) return rc;
  if (prob->density && !opt->sigma0_set) sp.s0 = graded_sigma0(opt->scheme, sp.s1);
  std::lock_guard<std::mutex> lk(g_mutex);
  hipStream_t st = reinterpret_cast<hipStream_t>(opt->stream);
  Plan* p = nullptr;
  const bool acc = sp.kind == K_ACC_EM || sp.kind == K_ACC_MS;
  scfft_options o = *opt;
  o.tol = -1;
  o.max_iter = iters + 1;
  SolveCtl c;
  SolveCoef cf;
  fill_ctl(c, o, sp.kind, prob->d, prob->e0);
  fill_coef(cf, sp, prob->density != nullptr, prob->d, prob->e0, (double)voxels(prob));
  const TuneCtx tc{map_kind(sp.kind, prob->density != nullptr), &c, &cf, prob->phase,
                   prob->density};
  rc = get_plan(prob->d, prob->n, opt->precision, 1, acc, opt->symbol, st, &p, 0,
                real_ok(sp, prob->d, prob->n, opt->precision), &tc);
  if (rc != SCFFT_OK) return rc;
  rc = ensure_hist(p, iters + 2);
  if (rc != SCFFT_OK) return rc;
  p->mk = tc.mk;
  SCFFT_HIP(hipMemcpyAsync(p->ctl, &c, sizeof(c), hipMemcpyHostToDevice, st));
  SCFFT_HIP(hipMemcpyAsync(p->coef, &cf, sizeof(cf), hipMemcpyHostToDevice, st));
  rc = launch_init(p, st);
  if (rc != SCFFT_OK) return rc;
  hipEvent_t ev[10];
  for (auto& e : ev) SCFFT_HIP(hipEventCreate(&e));
  double acc_ms[5] = {0, 0, 0, 0, 0};
  for (int it = 0; it < iters; ++it) {
    rc = launch_iteration(p, prob->phase, prob->density, st, true, ev);
    if (rc != SCFFT_OK) break;
    SCFFT_HIP(hipEventSynchronize(ev[p->d == 3 ? 9 : 7]));
    const int pairs[5][2] = {{0, 1}, {6, 7}, {4, 5}, {8, 9}, {2, 3}};
    for (int k = 0; k < 5; ++k) {
      if (p->d == 2 && (k == 2 || k == 3)) continue;
      float t = 0;
      SCFFT_HIP(hipEventElapsedTime(&t, ev[pairs[k][0]], ev[pairs[k][1]]));
      acc_ms[k] += t;
    }
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  for (int k = 0; k < 5; ++k) ms[k] = acc_ms[k] / iters;
  return rc;
}

}  // extern "C"

// ---------------------------------------------------- allocation-free solve
// scfft_solve_noalloc keeps its whole workspace in one file-scope device
// array.  Each GPU holds its own copy from the library's load until the
// process ends; host code reaches it only through the address that
// hipGetSymbolAddress reports for the current device (the array's name is a
// host-side stand-in, not a device address).
namespace scfft {
namespace {

constexpr size_t kScratchBytes = (size_t)SCFFT_NOALLOC_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct ScratchDev {
  unsigned char* ptr = nullptr;   // this device's copy of `scratch`
  hipEvent_t ev[2] = {nullptr, nullptr};
};
std::map<int, ScratchDev> g_scratch;   // guarded by g_mutex

// Set-up, once per device, with that device current.
scfft_status scratch_for_device(int dev, ScratchDev** out) {
  auto it = g_scratch.find(dev);
  if (it == g_scratch.end()) {
    ScratchDev sd;
    void* ptr = nullptr;
    SCFFT_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return SCFFT_ERR_DEVICE;
    sd.ptr = static_cast<unsigned char*>(ptr);
    SCFFT_HIP(hipEventCreate(&sd.ev[0]));
    SCFFT_HIP(hipEventCreate(&sd.ev[1]));
    it = g_scratch.emplace(dev, sd).first;
  }
  *out = &it->second;
  return SCFFT_OK;
}

// Points the plan's buffers into the block at base (256-byte aligned
// pieces); base == nullptr only sizes them.  Returns the bytes used.
size_t carve(Plan* p, unsigned char* base, int hist_cap) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    off = (off + 255) / 256 * 256;
    void* q = base ? static_cast<void*>(base + off) : nullptr;
    off += bytes;
    return q;
  };
  const size_t ns = (size_t)p->nsolve;
  p->X = take(p->xbytes);
  p->Ep = take(p->rbytes);
  if (p->st) {
    p->S = take(p->rbytes);
    p->T = take(p->rbytes);
  }
  p->part = static_cast<double*>(take(sizeof(double) * 5 * ns * p->d * p->xblocks));
  p->ctl = static_cast<SolveCtl*>(take(sizeof(SolveCtl) * ns));
  p->coef = static_cast<SolveCoef*>(take(sizeof(SolveCoef) * ns));
  p->hist_r = static_cast<double*>(take(sizeof(double) * (size_t)hist_cap * ns));
  p->hist_s = static_cast<double*>(take(2 * sizeof(double) * (size_t)hist_cap * ns));
  p->hist_cap = hist_cap;
  for (int a = 0; a < p->d; ++a) {
    p->tw[a] = take(p->esz * p->n[a]);
    p->sym[a] = static_cast<double*>(take(2 * sizeof(double) * p->n[a]));
  }
  return off;
}

}  // namespace
}  // namespace scfft

extern "C" {

scfft_status scfft_solve_noalloc(const scfft_problem* prob, const scfft_options* opt,
                                 scfft_result* res) {
  if (!res) return SCFFT_ERR_INVALID_ARG;
  if (!prob) return SCFFT_ERR_INVALID_ARG;
  SolveSpec sp{};
  scfft_status rc = prepare(prob, opt, cd(prob->sigma1.re, prob->sigma1.im), &sp);
  if (rc != SCFFT_OK) {
    res->status = rc;
    return rc;
  }
  if (prob->density && !opt->sigma0_set) sp.s0 = graded_sigma0(opt->scheme, sp.s1);
  std::lock_guard<std::mutex> lk(g_mutex);
  hipStream_t st = reinterpret_cast<hipStream_t>(opt->stream);
  int dev = 0;
  SCFFT_HIP(hipGetDevice(&dev));
  ScratchDev* sd = nullptr;
  rc = scratch_for_device(dev, &sd);
  if (rc != SCFFT_OK) return rc;
  Plan p;
  p.no_alloc = true;
  const bool acc = sp.kind == K_ACC_EM || sp.kind == K_ACC_MS;
  const bool real = real_ok(sp, prob->d, prob->n, opt->precision);
  // the knobs scfft_solve tuned for this configuration, if any (tuning itself
  // would allocate)
  bool tuned = false;
  const Knobs kn = cached_knobs(dev, prob->d, prob->n, opt->precision, acc, opt->symbol, real,
                                map_kind(sp.kind, prob->density != nullptr), &tuned);
  plan_shape(&p, dev, prob->d, prob->n, opt->precision, 1, acc, opt->symbol, real, kn);
  p.tuned = tuned;
  const int cap = opt->max_iter + 1;
  if (carve(&p, nullptr, cap) > kScratchBytes) {
    res->status = SCFFT_ERR_INVALID_ARG;
    return SCFFT_ERR_INVALID_ARG;
  }
  carve(&p, sd->ptr, cap);
  rc = plan_tables(&p, st);
  if (rc != SCFFT_OK) return rc;
  SolveCtl c;
  SolveCoef cf;
  fill_ctl(c, *opt, sp.kind, prob->d, prob->e0);
  fill_coef(cf, sp, prob->density != nullptr, prob->d, prob->e0, (double)p.M);
  p.mk = map_kind(sp.kind, prob->density != nullptr);
  SCFFT_HIP(hipMemcpyAsync(p.ctl, &c, sizeof(c), hipMemcpyHostToDevice, st));
  SCFFT_HIP(hipMemcpyAsync(p.coef, &cf, sizeof(cf), hipMemcpyHostToDevice, st));
  rc = launch_init(&p, st);
  if (rc != SCFFT_OK) return rc;
  double ms = 0;
  rc = run_loop({&p}, {prob->phase}, {prob->density}, opt->max_iter, opt->check_every, st, &ms,
                false, sd->ev);
  if (rc != SCFFT_OK) return rc;
  return read_result(&p, 0, prob, res, st, ms);
}

}  // extern "C"
