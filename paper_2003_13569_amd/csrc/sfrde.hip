// libsfrde: host plan, step drivers and the C ABI declared in include/sfrde.h.
//
// A plan holds, on the device: per-axis transform data (matrix-core
// fragments, FFT twiddles or dense matrices, built in FP64 on the host from
// the closed forms of Section 3.1), per-axis FP64
// eigenvalue tables, the six coefficient tables of the Alg. 1 precompute
// (computed in FP64 on the device, stored in dtype), and the workspace of the
// step: one field buffer P that every kernel transforms in place, and the
// retained spectral arrays u_hat, c_til, acc. The backward pass adds the
// adjoint buffers, a segment store for recomputed stage data and the
// derivative tables.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <cstdint>
#include <initializer_list>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/sfrde.h"
#include "coef.h"
#include "fft.h"
#include "kernels.h"
#include "mfma.h"
#include "stability.h"

using namespace sfrde;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHECK(expr)                                                                  \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(e_ == hipErrorOutOfMemory ? SFRDE_ENOMEM : SFRDE_EDEVICE, "%s: %s (%s:%d)", \
                  #expr, hipGetErrorString(e_), __FILE__, __LINE__);                    \
  } while (0)

#define TRY(expr)              \
  do {                         \
    int rc_ = (expr);          \
    if (rc_ != SFRDE_OK) return rc_; \
  } while (0)

const long long CKPT_MAGIC = 0x5346524445434b31LL;  // "SFRDECK1"
constexpr int MAX_N = 1024;
constexpr int MAX_BATCH = 65535;  // ensemble members: the launch's grid y extent
// Reduction scratch of the backward pass: per-block partials first, then the
// results of each ensemble member (2 S kappa/alpha sums, then parameters).
constexpr long long RED_OUT = 2 * MAX_SPECIES * 1024 + 64;
constexpr long long RED_PER_MEMBER = 2 * MAX_SPECIES + MAX_PARAMS;

// Device memory of sfrde_backward_noalloc: one array per GPU the library
// runs on, held until the process ends. Host code never passes `scratch`
// itself (in host code the name is a stand-in, not a device address): it
// uses the address hipGetSymbolAddress returns on each device, looked up
// once per device at plan set-up.
constexpr size_t SCRATCH_BYTES = (size_t)SFRDE_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// Address of this device's scratch array (the device must be current).
int scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= MAX_DEVICES) return fail(SFRDE_EDEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(SFRDE_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                  hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return SFRDE_OK;
}

}  // namespace

struct sfrde_plan_s {
  int ndim = 0;
  long long n[3] = {1, 1, 1};
  int bc = 0;
  double h[3] = {1, 1, 1};
  int S = 0;
  double alpha[MAX_SPECIES] = {0};  // member 0
  double kappa[MAX_SPECIES] = {0};
  double dt = 0;
  Rxn rxn{};
  // ensembles: B members of this grid; per-member orders, coefficients and
  // reaction constants ([B][S], [B])
  int B = 1;
  std::vector<double> alpha_m, kappa_m;
  std::vector<Rxn> rxn_m;
  Rxn* rxm = nullptr;  // device copy of rxn_m
  int dtype = 0;
  int scheme = 0;
  hipStream_t stream = nullptr;
  long long total = 0;
  double cs = 1;  // product of per-axis inverse scales
  size_t w = 4;   // bytes per real
  Geom geom[3]{};
  size_t lds[3] = {0, 0, 0};
  // matrix-core variant per axis (see mfma.h)
  bool use_m[3] = {false, false, false};
  // long periodic axes of 256, 512 or 1024 points: FFT tile kernels (fft.h)
  bool use_f[3] = {false, false, false};
  Geom geom_f[3]{};
  size_t lds_f[3] = {0, 0, 0};
  unsigned thr_f[3] = {0, 0, 0};
  void* tw[3] = {nullptr, nullptr, nullptr};  // [N][2] cos, sin of 2 pi m / N
  Geom geom_m[3]{};
  size_t lds_m[3] = {0, 0, 0};
  unsigned grid_m[3] = {0, 0, 0};
  MfmaAxisDev mfax[3]{};
  void* mf_A[3] = {nullptr, nullptr, nullptr};
  int n_cu = 256;
  int device = 0;
  // the static scratch array of the plan's device (allocation-free backward)
  void* scratch = nullptr;
  bool noalloc = false;  // this backward call carves its buffers from scratch
  // device memory
  void* Mt[3] = {nullptr, nullptr, nullptr};
  double* lam[3] = {nullptr, nullptr, nullptr};
  void* coef = nullptr;
  void* dcoef = nullptr;
  void* ltab = nullptr;  // P13 plans: L per species and point
  bool lfly = false;     // FP32 P13 Z kernels form L from the eigenvalues
  double* thp = nullptr;  // adjoint kappa/alpha partials per Z block [4][grid]
  bool thp_on = false;    // this backward call accumulates them (else G)
  size_t lam_off = 0;    // LDS byte offset of the eigenvalue tables (last axis kernels)
  void* P = nullptr;
  void* uhat = nullptr;
  void* ctil = nullptr;
  void* acc = nullptr;
  void* Pa = nullptr;
  void* zh = nullptr;
  void* aacc = nullptr;
  void* ahat = nullptr;
  void* gu = nullptr;
  double* G = nullptr;
  void* seg = nullptr;
  long long seg_steps = 0;   // steps the allocated segment store holds
  long long seg_cap = 0;     // its size in fields of [B][S][total]
  int seg_stride = 9;        // fields per step of the current backward (9, or 4 for u0 only)
  double* rp_acc = nullptr;
  double* red = nullptr;  // reduction scratch
  long long red_len = 0;
  int* flag = nullptr;
  int* h_flag = nullptr;  // pinned host mirror
  size_t bytes = 0;
  // measurement: optional HIP events around every kernel launch
  bool prof = false;
  std::vector<hipEvent_t> ev;    // start/stop pairs
  std::vector<int> ev_class;     // kernel class per pair
  size_t ev_used = 0;            // pairs recorded since the last reset
};

namespace {

// Elements and bytes of one field of every member: [B][S][total].
size_t field_elems(const sfrde_plan_s* p) { return (size_t)p->B * p->S * p->total; }
size_t field_bytes(const sfrde_plan_s* p) { return field_elems(p) * p->w; }

int dev_alloc(sfrde_plan_s* p, void** ptr, size_t bytes) {
  if (*ptr) return SFRDE_OK;
  hipError_t e = hipMalloc(ptr, bytes);
  if (e != hipSuccess) {
    *ptr = nullptr;
    return fail(e == hipErrorOutOfMemory ? SFRDE_ENOMEM : SFRDE_EDEVICE,
                "hipMalloc(%zu bytes): %s", bytes, hipGetErrorString(e));
  }
  p->bytes += bytes;
  return SFRDE_OK;
}

void dev_free(sfrde_plan_s* p, void** ptr, size_t bytes) {
  if (*ptr) {
    (void)hipFree(*ptr);
    p->bytes -= bytes;
    *ptr = nullptr;
  }
}

// Kernel classes for measurement (enum order of SFRDE_K_* in sfrde.h).
enum { KC_X = 0, KC_Y = 1, KC_Z = 2, KC_XADJ = 3, KC_ZADJ = 4, KC_OTHER = 5, KC_COUNT = 6 };

// Record the start event of a measured launch; returns the pair index or -1.
long long prof_start(sfrde_plan_s* p, int cls) {
  if (!p->prof) return -1;
  const size_t k = p->ev_used;
  while (p->ev.size() < 2 * (k + 1)) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return -1;
    p->ev.push_back(e);
  }
  if (p->ev_class.size() < k + 1) p->ev_class.resize(k + 1);
  p->ev_class[k] = cls;
  if (hipEventRecord(p->ev[2 * k], p->stream) != hipSuccess) return -1;
  p->ev_used = k + 1;
  return (long long)k;
}

void prof_stop(sfrde_plan_s* p, long long k) {
  if (k >= 0) (void)hipEventRecord(p->ev[2 * k + 1], p->stream);
}

int expected_nparams(int reaction, int S) {
  switch (reaction) {
    case RXN_LINEAR: return S;
    case RXN_FHN: return 5;
    case RXN_GRAY_SCOTT: return 2;
    case RXN_SCHNAKENBERG: return 3;
    case RXN_GM: return 5;
    case RXN_HUXLEY_MMS:
    case RXN_FISHER_MMS: return 0;
    default: return -1;
  }
}

// Transposed axis matrix Mt[j*n + k] = M[k][j] in FP64 (see kernels.h).
std::vector<double> axis_matrix_t(int bc, long long n) {
  const double pi = 3.14159265358979323846;
  std::vector<double> Mt((size_t)n * n);
  if (n == 1) {  // the one-point padding axis of a 1D plan: the identity
    Mt[0] = 1.0;
    return Mt;
  }
  for (long long k = 0; k < n; ++k) {
    for (long long j = 0; j < n; ++j) {
      double v;
      if (bc == SFRDE_BC_PERIODIC) {
        const long long N = n;
        const long long m = (k * j) % N;
        const double th = 2.0 * pi * double(m) / double(N);
        v = cos(th) + sin(th);
      } else if (bc == SFRDE_BC_DIRICHLET) {
        const long long N = n + 1;
        const long long m = ((k + 1) * (j + 1)) % (2 * N);
        v = sin(pi * double(m) / double(N));
      } else {
        const long long N = n - 1;
        const long long m = (k * j) % (2 * N);
        v = cos(pi * double(m) / double(N));
        if (j == 0 || j == n - 1) v *= 0.5;
      }
      Mt[(size_t)j * n + k] = v;
    }
  }
  return Mt;
}

double axis_inverse_scale(int bc, long long n) {
  if (n == 1) return 1.0;  // padding axis of a 1D plan
  if (bc == SFRDE_BC_PERIODIC) return 1.0 / double(n);
  if (bc == SFRDE_BC_DIRICHLET) return 2.0 / double(n + 1);
  return 2.0 / double(n - 1);
}

// log2(x) for a power of two x >= 1, else -1.
int pow2_shift(long long x) {
  if (x < 1 || (x & (x - 1)) != 0) return -1;
  int k = 0;
  while ((1LL << k) < x) ++k;
  return k;
}

long long pow2_floor(long long x) {
  long long p = 1;
  while (p * 2 <= x) p *= 2;
  return p;
}

void make_geom(sfrde_plan_s* p, int axis, long long min_tiles = 0) {
  Geom& g = p->geom[axis];
  const long long n = p->n[axis];
  long long inner = 1;
  for (int a = 0; a < axis; ++a) inner *= p->n[a];
  g.n = (int)n;
  g.spt = p->S;
  g.fast = 0;
  g.inner = inner;
  g.total = p->total;
  // Tile width: a power of two with n*W <= KMAX*NTHREADS, the tile of all
  // species within 64 KB of LDS, and no wider than the lines available.
  long long W = std::min<long long>(64, pow2_floor(std::max<long long>(1, (KMAX * NTHREADS) / n)));
  while (W > 1 && (size_t)p->S * n * (W + 1) * p->w > 65536) W /= 2;
  if (inner > 1) W = std::min<long long>(W, pow2_floor(inner) * (pow2_floor(inner) < inner ? 2 : 1));
  // Narrower tiles where there are too few lines to fill the device (small
  // grids, e.g. 2D): the dense kernels run one tile per block.
  auto tiles_for = [&](long long w) {
    const long long lines = p->total / n;
    return inner == 1 ? (lines + w - 1) / w : (p->total / (n * inner)) * ((inner + w - 1) / w);
  };
  while (W > 1 && tiles_for(W) < min_tiles) W /= 2;
  g.W = (int)W;
  g.pitch = (int)(W + 1);
  g.wshift = 0;
  while ((1 << g.wshift) < g.W) ++g.wshift;
  g.inv_n = 1.0f / (float)n;
  if (inner == 1) {
    g.outer = p->total / n;
    g.tpo = 1;
    g.tposh = 0;
    g.ntiles = (g.outer + W - 1) / W;
  } else {
    g.outer = p->total / (n * inner);
    g.tpo = (inner + W - 1) / W;
    g.tposh = pow2_shift(g.tpo);
    g.ntiles = g.outer * g.tpo;
  }
  size_t tile = (size_t)p->S * n * g.pitch * p->w;
  p->lds[axis] = std::max<size_t>(tile, NTHREADS * sizeof(double));
}

// ------------------------------------------------------------------ matrix cores
// Folded form of one axis matrix (mfma.h): the half matrices E and O over the
// fold pairs (the same pairs fold_pair() computes on the device), from which
// the fragment-ordered copies the waves load into registers are made.
struct MfmaTables {
  bool ok = false;
  int hK = 0, RBe = 0, RB = 0, ns = 0, rowsE = 0, rowsO = 0;
  std::vector<double> E, O;  // [rows][hK]
};

double axis_entry(int bc, long long n, long long k, long long j) {
  const double pi = 3.14159265358979323846;
  if (bc == SFRDE_BC_DIRICHLET) {
    const long long N = n + 1;
    return sin(pi * double(((k + 1) * (j + 1)) % (2 * N)) / double(N));
  }
  const long long N = n - 1;  // Neumann
  double v = cos(pi * double((k * j) % (2 * N)) / double(N));
  if (j == 0 || j == n - 1) v *= 0.5;
  return v;
}

MfmaTables mfma_tables(int bc, long long n) {
  const double pi = 3.14159265358979323846;
  MfmaTables t;
  std::vector<std::pair<long long, long long>> pairs;  // (a, b), b = -1: fixed point
  if (bc == SFRDE_BC_PERIODIC) {
    const long long N = n;
    pairs.push_back({0, -1});
    for (long long j = 1; j < (N + 1) / 2; ++j) pairs.push_back({j, N - j});
    if (N % 2 == 0) pairs.push_back({N / 2, -1});
    t.rowsE = (int)(N / 2 + 1);
    t.rowsO = t.rowsE;
  } else {
    for (long long j = 0; j < n / 2; ++j) pairs.push_back({j, n - 1 - j});
    if (n % 2 == 1) pairs.push_back({(n - 1) / 2, -1});
    t.rowsE = (int)((n + 1) / 2);
    t.rowsO = (int)(n / 2);
  }
  t.ns = (int)pairs.size();
  t.hK = ((t.ns + 31) / 32) * 32;
  t.RBe = (t.rowsE + 15) / 16;
  t.RB = t.RBe + (t.rowsO + 15) / 16;
  t.ok = t.hK <= 128 && t.RB <= MF_WAVES;
  if (!t.ok) return t;
  t.E.assign((size_t)t.rowsE * t.hK, 0.0);
  t.O.assign((size_t)t.rowsO * t.hK, 0.0);
  for (int i = 0; i < t.ns; ++i) {
    const long long a = pairs[i].first;
    const bool fixed = pairs[i].second < 0;
    for (int m = 0; m < t.rowsE; ++m) {
      double e, o;
      if (bc == SFRDE_BC_PERIODIC) {
        const double th = 2.0 * pi * double((m * a) % n) / double(n);
        e = cos(th);
        o = fixed ? 0.0 : sin(th);
      } else {
        e = axis_entry(bc, n, 2 * m, a);
        o = (fixed || m >= t.rowsO) ? 0.0 : axis_entry(bc, n, 2 * m + 1, a);
      }
      t.E[(size_t)m * t.hK + i] = e;
      if (m < t.rowsO) t.O[(size_t)m * t.hK + i] = o;
    }
  }
  return t;
}

// binary16 bits of x rounded to nearest even (subnormals included; |x| is
// far below the binary16 maximum here).
unsigned short host_f16(double x) {
  const unsigned short sign = std::signbit(x) ? 0x8000 : 0;
  const double a = std::fabs(x);
  if (a <= std::ldexp(1.0, -25)) return sign;  // 2^-25 is the tie with 0
  int e;
  std::frexp(a, &e);  // a in [2^(e-1), 2^e)
  int E = std::max(e - 1, -14);
  double m = std::nearbyint(a / std::ldexp(1.0, E - 10));
  if (m >= 2048.0) {
    m *= 0.5;
    E += 1;
  }
  if (m < 1024.0) return (unsigned short)(sign | (unsigned)m);  // subnormal
  return (unsigned short)(sign | ((unsigned)(E + 15) << 10) | ((unsigned)m - 1024u));
}
double host_f16_value(unsigned short h) {
  const int ex = (h >> 10) & 31, man = h & 1023;
  const double v = ex == 0 ? std::ldexp((double)man, -24) : std::ldexp((double)(man + 1024), ex - 25);
  return (h & 0x8000) ? -v : v;
}

double half_entry(const MfmaTables& t, int rb, int row16, int k) {
  const bool isE = rb < t.RBe;
  const int row = 16 * (isE ? rb : rb - t.RBe) + row16;
  const int rows = isE ? t.rowsE : t.rowsO;
  if (row >= rows || k >= t.hK) return 0.0;
  return isE ? t.E[(size_t)row * t.hK + k] : t.O[(size_t)row * t.hK + k];
}

int setup_mfma_axis(sfrde_plan_s* p, int axis) {
  if (p->n[axis] < 2) return SFRDE_OK;  // padding axis of a 1D plan: dense kernels
  MfmaTables t = mfma_tables(p->bc, p->n[axis]);
  if (!t.ok) return SFRDE_OK;
  const bool f32 = p->dtype == SFRDE_F32;
  const int W = f32 ? (axis == 0 ? XfX<float>::W : XfZ<float>::W) : MfmaXfF64::W;
  const int threads = f32 ? XfZ<float>::THREADS : MfmaXfF64::THREADS;
  // geometry
  Geom& g = p->geom_m[axis];
  g = p->geom[axis];
  g.W = W;
  g.pitch = W + 1;
  g.wshift = 0;
  while ((1 << g.wshift) < g.W) ++g.wshift;
  if (g.inner == 1) {
    g.tpo = 1;
    g.tposh = 0;
    g.ntiles = (g.outer + W - 1) / W;
  } else {
    // Tiles along strided axes hold one species (the species index becomes
    // part of the outer block index; the fields are [S][total]): always in
    // FP32, whose vector paths assume it, and in FP64 when the launch (all
    // members) split by species still has at most one block per CU, i.e.
    // leaves CUs idle otherwise; FP64 tiles of every species are faster
    // once the blocks outnumber the CUs.
    const long long tiles_all = g.outer * ((g.inner + W - 1) / W) * p->B;
    if (f32 || tiles_all * p->S <= (long long)p->n_cu) {
      g.outer *= p->S;
      g.spt = 1;
    }
    g.tpo = (g.inner + W - 1) / W;
    g.tposh = pow2_shift(g.tpo);
    g.ntiles = g.outer * g.tpo;
  }
  // vector tile paths of the FP32 engine (their thread layouts assume these)
  if (f32 && g.inner == 1)
    g.fast = (g.n == 64 || g.n == 128 || g.n == 256) && (long long)p->S * g.n <= 512 &&
             (long long)p->S * g.n >= 64 && g.outer % W == 0;
  else if (f32)
    g.fast = g.inner % W == 0 && g.n % 64 == 0 && g.n <= 256;
  else  // FP64: full tiles of at most two species move through registers (TileIOF64;
        // its x-axis layout needs n = 64, 128 or 256, strided axes a multiple of 64)
    g.fast = g.n % 64 == 0 && g.n <= 256 && g.spt <= 2 &&
             (g.inner == 1 ? g.outer % W == 0 && (g.n & (g.n - 1)) == 0 : g.inner % W == 0);
  MfmaAxisDev& ax = p->mfax[axis];
  ax.hK = t.hK;
  ax.RBe = t.RBe;
  ax.RB = t.RB;
  ax.fb_pitch = p->dtype == SFRDE_F32 ? F32_FBP : t.hK + 2;
  ax.r_pitch = W + 1;
  ax.direct = p->bc != SFRDE_BC_PERIODIC;
  size_t tile_bytes = (size_t)g.spt * g.n * g.pitch * p->w;
  tile_bytes = (tile_bytes + 15) / 16 * 16;
  // fold area: FP32 plans keep two binary16 terms of s and d and the column
  // scales; FP64 plans s and d.
  const size_t fold_bytes = p->dtype == SFRDE_F32 ? (size_t)f32_fold_bytes(W)
                                                   : (size_t)2 * W * ax.fb_pitch * 8;
  const size_t res_bytes = (size_t)16 * t.RB * ax.r_pitch * p->w;
  ax.fb_off = (int)tile_bytes;
  // FP32 x tiles: a second fold buffer where it fits (the unfold's result
  // rows fit one buffer)
  ax.nfb = p->dtype == SFRDE_F32 && axis == 0 &&
                   tile_bytes + std::max(2 * fold_bytes, res_bytes) <= 160 * 1024
               ? 2
               : 1;
  size_t lds = tile_bytes + std::max(ax.nfb * fold_bytes, res_bytes);
  lds = std::max<size_t>(lds, (size_t)threads * sizeof(double));
  if (lds > 160 * 1024) return SFRDE_OK;  // does not fit: FFT or dense kernels
  // the engine's tile indices are 32-bit, with room for one stride of the grid
  if (g.ntiles > 0x7fff0000LL) return SFRDE_OK;
  p->lds_m[axis] = lds;
  // persistent grid: as many blocks as fit on the CUs at once
  const long long per_cu = 1;
  // ensembles launch B times these blocks (blockIdx.y = member)
  const long long slots = std::max<long long>(1, ((long long)p->n_cu * per_cu + p->B - 1) / p->B);
  p->grid_m[axis] = (unsigned)std::min<long long>(g.ntiles, slots);
  // fragment-ordered split matrices
  if (p->dtype == SFRDE_F32) {
    std::vector<unsigned short> frag((size_t)MF_WAVES * MF_KSMAX_F32 * 2 * 64 * 8, 0);
    for (int rb = 0; rb < t.RB; ++rb)
      for (int ks = 0; ks < MF_KSMAX_F32; ++ks)
        for (int lane = 0; lane < 64; ++lane)
          for (int e = 0; e < 8; ++e) {
            // folded entries 64 and up sit rotated by four within each group
            // of eight in the engine's fold buffer: the same order here
            const int k = 32 * ks + 8 * (lane / 16) + e;
            const double v = half_entry(t, rb, lane % 16, k >= 64 ? k ^ 4 : k);
            const unsigned short h0 = host_f16(v);
            const unsigned short h1 = host_f16(v - host_f16_value(h0));
            frag[((((size_t)rb * MF_KSMAX_F32 + ks) * 2 + 0) * 64 + lane) * 8 + e] = h0;
            frag[((((size_t)rb * MF_KSMAX_F32 + ks) * 2 + 1) * 64 + lane) * 8 + e] = h1;
          }
    TRY(dev_alloc(p, &p->mf_A[axis], frag.size() * sizeof(unsigned short)));
    HIPCHECK(hipMemcpy(p->mf_A[axis], frag.data(), frag.size() * sizeof(unsigned short),
                       hipMemcpyHostToDevice));
  } else {
    std::vector<double> frag((size_t)MF_WAVES * MF_KSMAX_F64 * 64, 0.0);
    for (int rb = 0; rb < t.RB; ++rb)
      for (int ks = 0; ks < MF_KSMAX_F64; ++ks)
        for (int lane = 0; lane < 64; ++lane)
          frag[((size_t)rb * MF_KSMAX_F64 + ks) * 64 + lane] =
              half_entry(t, rb, lane % 16, 4 * ks + lane / 16);
    TRY(dev_alloc(p, &p->mf_A[axis], frag.size() * sizeof(double)));
    HIPCHECK(hipMemcpy(p->mf_A[axis], frag.data(), frag.size() * sizeof(double),
                       hipMemcpyHostToDevice));
  }
  ax.Afrag = p->mf_A[axis];
  ax.n = (int)p->n[axis];
  ax.ns = t.ns;
  ax.periodic = p->bc == SFRDE_BC_PERIODIC;
  p->use_m[axis] = true;
  return SFRDE_OK;
}

// Long periodic axes of N = 256, 512 or 1024 points run the FFT tile kernels
// (fft.h): x tiles hold 2 lines of every species (1 line for S > 2), strided
// tiles 4 lines of one species, one wavefront per pair of lines.
template <typename T>
int setup_fft_axis(sfrde_plan_s* p, int axis) {
  const long long n = p->n[axis];
  if (p->use_m[axis] || p->bc != SFRDE_BC_PERIODIC ||
      !(n == 256 || n == 512 || n == 1024))
    return SFRDE_OK;
  Geom& g = p->geom_f[axis];
  g = p->geom[axis];
  if (g.inner == 1) {
    g.spt = p->S;
    g.W = p->S <= 2 ? 2 : 1;
    g.tpo = 1;
    g.tposh = 0;
    g.ntiles = (g.outer + g.W - 1) / g.W;
  } else {
    g.outer *= p->S;  // one species per tile: the species joins the outer index
    g.spt = 1;
    g.W = 4;
    g.tpo = (g.inner + g.W - 1) / g.W;
    g.tposh = pow2_shift(g.tpo);
    g.ntiles = g.outer * g.tpo;
  }
  g.pitch = g.W | 1;  // odd: a line's elements fall in distinct LDS banks
  g.wshift = 0;
  while ((1 << g.wshift) < g.W) ++g.wshift;
  g.fast = 0;
  p->thr_f[axis] = FFT_THREADS;  // >= 64 per line pair (at most 2 here)
  p->lds_f[axis] = fft_lds_bytes<T>(g.spt, g.n, g.W, g.pitch);
  if (p->lds_f[axis] > 160 * 1024) return SFRDE_OK;  // dense kernels
  const double pi = 3.14159265358979323846;
  std::vector<T> tw((size_t)2 * n);
  for (long long m = 0; m < n; ++m) {
    tw[2 * m] = T(cos(2.0 * pi * double(m) / double(n)));
    tw[2 * m + 1] = T(sin(2.0 * pi * double(m) / double(n)));
  }
  TRY(dev_alloc(p, &p->tw[axis], tw.size() * sizeof(T)));
  HIPCHECK(hipMemcpy(p->tw[axis], tw.data(), tw.size() * sizeof(T), hipMemcpyHostToDevice));
  std::vector<const void*> fns = {
      reinterpret_cast<const void*>(&k_xstage<T, FftXf, true>),
      reinterpret_cast<const void*>(&k_zstage<T, FftXf, true>),
      reinterpret_cast<const void*>(&k_xadj<T, FftXf, true>),
      reinterpret_cast<const void*>(&k_zadj<T, FftXf, true>),
      reinterpret_cast<const void*>(&k_single<T, FftXf, true>)};
  for (const void* f : fns)
    HIPCHECK(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)p->lds_f[axis]));
  p->use_f[axis] = true;
  return SFRDE_OK;
}

template <typename T>
int set_lds_attrs(size_t bytes) {
  std::vector<const void*> fns = {
      reinterpret_cast<const void*>(&k_xstage_m<T, XfX<T>, false>),
      reinterpret_cast<const void*>(&k_zstage_m<T, XfZ<T>, -1, false>),
      reinterpret_cast<const void*>(&k_zstage_m<T, XfZ<T>, 0, false>),
      reinterpret_cast<const void*>(&k_zstage_m<T, XfZ<T>, 1, false>),
      reinterpret_cast<const void*>(&k_zstage_m<T, XfZ<T>, 2, false>),
      reinterpret_cast<const void*>(&k_zstage_m<T, XfZ<T>, 3, false>),
      reinterpret_cast<const void*>(&k_xadj_m<T, XfX<T>, false>),
      reinterpret_cast<const void*>(&k_zadj_m<T, XfZ<T>, false>),
      reinterpret_cast<const void*>(&k_single_m<T, XfX<T>, false>),
      reinterpret_cast<const void*>(&k_single_m<T, XfZ<T>, false>)};
  if constexpr (std::is_same<T, double>::value) {
    const void* kinds[] = {
        reinterpret_cast<const void*>(&k_xadj_m<T, XfX<T>, false, 2, false, RXN_LINEAR>),
        reinterpret_cast<const void*>(&k_xadj_m<T, XfX<T>, false, 2, false, RXN_FHN>),
        reinterpret_cast<const void*>(&k_xadj_m<T, XfX<T>, false, 2, false, RXN_GRAY_SCOTT>),
        reinterpret_cast<const void*>(&k_xadj_m<T, XfX<T>, false, 2, false, RXN_SCHNAKENBERG>),
        reinterpret_cast<const void*>(&k_xadj_m<T, XfX<T>, false, 2, false, RXN_GM>)};
    for (const void* f : kinds) fns.push_back(f);
  }
  if constexpr (std::is_same<T, float>::value) {
    const void* fast[] = {reinterpret_cast<const void*>(&k_xstage_m<T, XfX<T>, true>),
                          reinterpret_cast<const void*>(&k_zstage_m<T, XfZ<T>, -1, true>),
                          reinterpret_cast<const void*>(&k_zstage_m<T, XfZ<T>, 0, true>),
                          reinterpret_cast<const void*>(&k_zstage_m<T, XfZ<T>, 1, true>),
                          reinterpret_cast<const void*>(&k_zstage_m<T, XfZ<T>, 2, true>),
                          reinterpret_cast<const void*>(&k_zstage_m<T, XfZ<T>, 3, true>),
                          reinterpret_cast<const void*>(&k_xadj_m<T, XfX<T>, true>),
                          reinterpret_cast<const void*>(&k_zadj_m<T, XfZ<T>, true>),
                          reinterpret_cast<const void*>(&k_zadj_m<T, XfZ<T>, true, 0, 0>),
                          reinterpret_cast<const void*>(&k_zadj_m<T, XfZ<T>, true, 1, 0>),
                          reinterpret_cast<const void*>(&k_zadj_m<T, XfZ<T>, true, 2, 0>),
                          reinterpret_cast<const void*>(&k_zadj_m<T, XfZ<T>, true, 3, 0>),
                          reinterpret_cast<const void*>(&k_zadj_m<T, XfZ<T>, true, MODE_INIT, 0>),
                          reinterpret_cast<const void*>(&k_zadj_m<T, XfZ<T>, true, 0, 1>),
                          reinterpret_cast<const void*>(&k_zadj_m<T, XfZ<T>, true, 1, 1>),
                          reinterpret_cast<const void*>(&k_zadj_m<T, XfZ<T>, true, 2, 1>),
                          reinterpret_cast<const void*>(&k_zadj_m<T, XfZ<T>, true, 3, 1>),
                          reinterpret_cast<const void*>(&k_zadj_m<T, XfZ<T>, true, MODE_INIT, 1>),
                          reinterpret_cast<const void*>(&k_xadj_m<T, XfX<T>, true, 1>),
                          reinterpret_cast<const void*>(&k_xadj_m<T, XfX<T>, true, 2>),
                          reinterpret_cast<const void*>(&k_xadj_m<T, XfX<T>, true, 2, true>),
                          reinterpret_cast<const void*>(&k_single_m<T, XfX<T>, true>),
                          reinterpret_cast<const void*>(&k_single_m<T, XfZ<T>, true>),
                          reinterpret_cast<const void*>(&k_single_m<T, XfZ<T>, true, 1>),
                          reinterpret_cast<const void*>(&k_single_m<T, XfX<T>, true, 2>),
                          reinterpret_cast<const void*>(&k_single_m<T, XfZ<T>, true, 2>),
                          reinterpret_cast<const void*>(&k_xstage_m<T, XfX<T>, true, RXN_LINEAR>),
                          reinterpret_cast<const void*>(&k_xstage_m<T, XfX<T>, true, RXN_FHN>),
                          reinterpret_cast<const void*>(&k_xstage_m<T, XfX<T>, true, RXN_GRAY_SCOTT>),
                          reinterpret_cast<const void*>(&k_xstage_m<T, XfX<T>, true, RXN_SCHNAKENBERG>),
                          reinterpret_cast<const void*>(&k_xstage_m<T, XfX<T>, true, RXN_GM>)};
    for (const void* f : fast) fns.push_back(f);
  }
  for (const void* f : fns)
    HIPCHECK(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  return SFRDE_OK;
}

// --------------------------------------------------------------------------
template <typename T>
StageArgs<T> stage_args(sfrde_plan_s* p, int axis, void* P) {
  StageArgs<T> a{};
  a.g = p->use_m[axis] ? p->geom_m[axis] : p->use_f[axis] ? p->geom_f[axis] : p->geom[axis];
  a.Mt = (const T*)(p->use_f[axis] ? p->tw[axis] : p->Mt[axis]);
  a.P = (T*)P;
  a.coef = (const T*)p->coef;
  a.ltab = (const T*)p->ltab;
  a.dcoef = (const T*)p->dcoef;
  a.tau = T(p->dt);
  for (int k = 0; k < 3; ++k) a.lam[k] = p->lam[k];
  for (int s = 0; s < p->S; ++s) {
    a.kt[s] = T(p->kappa[s] * p->dt);
    a.ha[s] = T(0.5 * p->alpha[s]);
  }
  a.lfly = p->lfly && axis == p->ndim - 1;
  a.lam_off = (int)p->lam_off;
  a.uhat = (T*)p->uhat;
  a.ctil = (T*)p->ctil;
  a.acc = (T*)p->acc;
  a.zh = (T*)p->zh;
  a.aacc = (T*)p->aacc;
  a.ahat = (T*)p->ahat;
  a.gu = (T*)p->gu;
  a.flag = p->flag;
  a.rxn = p->rxn;
  a.nmem = p->B;
  a.fsz = (long long)p->S * p->total;
  a.rxm = p->rxm;
  a.cs = T(p->cs);
  a.S = p->S;
  a.neumann = p->bc == SFRDE_BC_NEUMANN;
  a.n0 = p->n[0];
  a.n1 = p->n[1];
  a.n2 = p->n[2];
  return a;
}

// The FP32 engine's vector tile paths: the axis geometry allows them and
// every field pointer the kernel moves tiles of is 16-byte aligned.
template <typename T>
bool use_fast(const sfrde_plan_s* p, int axis, std::initializer_list<const void*> ptrs) {
  if (!std::is_same<T, float>::value || !p->geom_m[axis].fast) return false;
  for (const void* q : ptrs)
    if (reinterpret_cast<uintptr_t>(q) & 15u) return false;
  return true;
}

// FP64 matrix-core launches move tiles through registers only with 16-byte
// aligned fields (the plan's own buffers always are).
template <typename T>
void align_check(Geom& g, std::initializer_list<const void*> ptrs) {
  if (std::is_same<T, float>::value) return;
  for (const void* q : ptrs)
    if (reinterpret_cast<uintptr_t>(q) & 15u) g.fast = 0;
}

template <typename T>
int launch_single(sfrde_plan_s* p, int axis, const void* src, void* dst, int pre_div, int post_mul) {
  SingleArgs<T> a{};
  a.g = p->use_m[axis] ? p->geom_m[axis] : p->use_f[axis] ? p->geom_f[axis] : p->geom[axis];
  align_check<T>(a.g, {src, dst});
  a.Mt = (const T*)(p->use_f[axis] ? p->tw[axis] : p->Mt[axis]);
  a.src = (const T*)src;
  a.dst = (T*)dst;
  a.S = p->S;
  a.pre_divide_w = pre_div && p->bc == SFRDE_BC_NEUMANN;
  a.post_multiply_w = post_mul && p->bc == SFRDE_BC_NEUMANN;
  a.nmem = p->B;
  a.fsz = (long long)p->S * p->total;
  a.n0 = p->n[0];
  a.n1 = p->n[1];
  a.n2 = p->n[2];
  const long long pk = prof_start(p, KC_Y);
  if (p->use_m[axis]) {
    const dim3 grid(p->grid_m[axis], p->B);
    const size_t lds = p->lds_m[axis];
    const bool fast = use_fast<T>(p, axis, {src, dst});
    // fast launches without point weights: the kernel holding only the
    // tile path that runs
    const bool plain = fast && !a.pre_divide_w && !a.post_multiply_w;
    // results straight to global memory: DCT-I / DST-I on one-species
    // strided tiles (rows inner apart, columns contiguous)
    const bool to_glob = p->mfax[axis].direct != 0 && a.g.spt == 1 && a.g.inner > 1;
    if (axis == 0) {
      const dim3 block(XfX<T>::THREADS);
      if constexpr (std::is_same<T, float>::value)
        if (fast) {
          if (plain)  // x tiles: through the tile
            hipLaunchKernelGGL((k_single_m<T, XfX<T>, true, 2>), grid, block, lds, p->stream, a,
                               p->mfax[axis]);
          else
            hipLaunchKernelGGL((k_single_m<T, XfX<T>, true>), grid, block, lds, p->stream, a,
                               p->mfax[axis]);
          goto launched;
        }
      hipLaunchKernelGGL((k_single_m<T, XfX<T>, false>), grid, block, lds, p->stream, a,
                         p->mfax[axis]);
    } else {
      const dim3 block(XfZ<T>::THREADS);
      if constexpr (std::is_same<T, float>::value)
        if (fast) {
          if (plain && to_glob)
            hipLaunchKernelGGL((k_single_m<T, XfZ<T>, true, 1>), grid, block, lds, p->stream, a,
                               p->mfax[axis]);
          else if (plain)
            hipLaunchKernelGGL((k_single_m<T, XfZ<T>, true, 2>), grid, block, lds, p->stream, a,
                               p->mfax[axis]);
          else
            hipLaunchKernelGGL((k_single_m<T, XfZ<T>, true>), grid, block, lds, p->stream, a,
                               p->mfax[axis]);
          goto launched;
        }
      hipLaunchKernelGGL((k_single_m<T, XfZ<T>, false>), grid, block, lds, p->stream, a,
                         p->mfax[axis]);
    }
  } else if (p->use_f[axis]) {
    hipLaunchKernelGGL((k_single<T, FftXf, true>), dim3((unsigned)a.g.ntiles, p->B),
                       dim3(p->thr_f[axis]), p->lds_f[axis], p->stream, a);
  } else
    hipLaunchKernelGGL(k_single<T>, dim3((unsigned)a.g.ntiles, p->B), dim3(NTHREADS),
                       p->lds[axis], p->stream, a);
launched:
  prof_stop(p, pk);
  HIPCHECK(hipGetLastError());
  return SFRDE_OK;
}

// Stored data of one step inside the segment store.
template <typename T>
struct StepStore {
  T* phys;  // [B][4][S][total]
  T* uhat;  // [B][S][total]
  T* fhat;  // [B][4][S][total]
};

template <typename T>
StepStore<T> step_store(sfrde_plan_s* p, long long slot) {
  StepStore<T> s{nullptr, nullptr, nullptr};
  if (!p->seg) return s;
  const size_t f = field_elems(p);
  T* base = (T*)p->seg + (size_t)slot * p->seg_stride * f;
  s.phys = base;
  if (p->seg_stride == 9) {  // u_hat and the four f_hat: the kappa/alpha terms
    s.uhat = base + 4 * f;
    s.fhat = base + 5 * f;
  }
  return s;
}

template <typename T>
int launch_x(sfrde_plan_s* p, int stage, double t, T* st_phys) {
  StageArgs<T> a = stage_args<T>(p, 0, p->P);
  a.mode = stage;
  a.t = t;
  a.st_phys = st_phys;
  const long long pk = prof_start(p, KC_X);
  if (p->use_m[0]) {
    const dim3 grid(p->grid_m[0], p->B), block(XfX<T>::THREADS);
    const bool fast = use_fast<T>(p, 0, {p->P, st_phys});
    // FP32, two species, non-periodic x: the register-fed kernel of the
    // plan's reaction kind
    const int rk = std::is_same<T, float>::value && fast && p->S == 2 &&
                           p->bc != SFRDE_BC_PERIODIC && p->rxn.kind <= RXN_GM
                       ? p->rxn.kind
                       : -1;
    if constexpr (std::is_same<T, float>::value) {
      if (rk >= 0) {
        const size_t lds = p->lds_m[0];
        switch (rk) {
          case RXN_LINEAR: hipLaunchKernelGGL((k_xstage_m<T, XfX<T>, true, RXN_LINEAR>), grid, block, lds, p->stream, a, p->mfax[0]); break;
          case RXN_FHN: hipLaunchKernelGGL((k_xstage_m<T, XfX<T>, true, RXN_FHN>), grid, block, lds, p->stream, a, p->mfax[0]); break;
          case RXN_GRAY_SCOTT: hipLaunchKernelGGL((k_xstage_m<T, XfX<T>, true, RXN_GRAY_SCOTT>), grid, block, lds, p->stream, a, p->mfax[0]); break;
          case RXN_SCHNAKENBERG: hipLaunchKernelGGL((k_xstage_m<T, XfX<T>, true, RXN_SCHNAKENBERG>), grid, block, lds, p->stream, a, p->mfax[0]); break;
          default: hipLaunchKernelGGL((k_xstage_m<T, XfX<T>, true, RXN_GM>), grid, block, lds, p->stream, a, p->mfax[0]); break;
        }
        goto x_launched;
      }
    }
    if (fast)
      hipLaunchKernelGGL((k_xstage_m<T, XfX<T>, std::is_same<T, float>::value>), grid, block,
                         p->lds_m[0], p->stream, a, p->mfax[0]);
    else
      hipLaunchKernelGGL((k_xstage_m<T, XfX<T>, false>), grid, block, p->lds_m[0], p->stream, a,
                         p->mfax[0]);
  x_launched:;
  } else if (p->use_f[0]) {
    hipLaunchKernelGGL((k_xstage<T, FftXf, true>), dim3((unsigned)a.g.ntiles, p->B), dim3(p->thr_f[0]),
                       p->lds_f[0], p->stream, a);
  } else
    hipLaunchKernelGGL(k_xstage<T>, dim3((unsigned)a.g.ntiles, p->B), dim3(NTHREADS),
                       p->lds[0], p->stream, a);
  prof_stop(p, pk);
  HIPCHECK(hipGetLastError());
  return SFRDE_OK;
}

// The four forward stages of FP32 plans have their own Z kernels.
template <typename T>
void launch_zstage_m(bool fast, int mode, dim3 grid, size_t lds, hipStream_t st,
                     const StageArgs<T>& a, const MfmaAxisDev& ax) {
  const dim3 block(XfZ<T>::THREADS);
  if constexpr (std::is_same<T, float>::value) {
    if (fast) {
      switch (mode) {
        case 0: hipLaunchKernelGGL((k_zstage_m<T, XfZ<T>, 0, true>), grid, block, lds, st, a, ax); return;
        case 1: hipLaunchKernelGGL((k_zstage_m<T, XfZ<T>, 1, true>), grid, block, lds, st, a, ax); return;
        case 2: hipLaunchKernelGGL((k_zstage_m<T, XfZ<T>, 2, true>), grid, block, lds, st, a, ax); return;
        case 3: hipLaunchKernelGGL((k_zstage_m<T, XfZ<T>, 3, true>), grid, block, lds, st, a, ax); return;
        default: hipLaunchKernelGGL((k_zstage_m<T, XfZ<T>, -1, true>), grid, block, lds, st, a, ax); return;
      }
    }
  }
  if constexpr (!std::is_same<T, float>::value) {
    switch (mode) {
      case 0: hipLaunchKernelGGL((k_zstage_m<T, XfZ<T>, 0, false>), grid, block, lds, st, a, ax); return;
      case 1: hipLaunchKernelGGL((k_zstage_m<T, XfZ<T>, 1, false>), grid, block, lds, st, a, ax); return;
      case 2: hipLaunchKernelGGL((k_zstage_m<T, XfZ<T>, 2, false>), grid, block, lds, st, a, ax); return;
      case 3: hipLaunchKernelGGL((k_zstage_m<T, XfZ<T>, 3, false>), grid, block, lds, st, a, ax); return;
      default: break;
    }
  }
  hipLaunchKernelGGL((k_zstage_m<T, XfZ<T>, -1, false>), grid, block, lds, st, a, ax);
}

// uhat: the spectral state this stage reads (stages 0, 1) or writes (stage
// 3); NULL: the plan's own.
template <typename T>
int launch_z(sfrde_plan_s* p, int mode, const void* src, T* st_fhat, T* uhat = nullptr) {
  const int ax = p->ndim - 1;
  StageArgs<T> a = stage_args<T>(p, ax, p->P);
  a.mode = mode;
  a.src = (const T*)src;
  align_check<T>(a.g, {src});
  a.st_fhat = st_fhat;
  if (uhat) a.uhat = uhat;
  const long long pk = prof_start(p, KC_Z);
  if (p->use_m[ax])
    {
      const bool fast = use_fast<T>(p, ax, {p->P, src});
      // the per-stage kernels: forward stages (the vector layout holds last
      // axes of 64 to 256 points in steps of 64), L formed in the kernel or
      // read from the table
      const bool staged = fast && mode >= 0 && mode <= 3 && !src && (p->lfly || p->ltab);
      launch_zstage_m<T>(fast, staged || (!fast && !src && mode >= 0 && mode <= 3) ? mode : -1,
                         dim3(p->grid_m[ax], p->B), p->lds_m[ax], p->stream, a, p->mfax[ax]);
    }
  else if (p->use_f[ax]) {
    hipLaunchKernelGGL((k_zstage<T, FftXf, true>), dim3((unsigned)a.g.ntiles, p->B), dim3(p->thr_f[ax]),
                       p->lds_f[ax], p->stream, a);
  } else
    hipLaunchKernelGGL(k_zstage<T>, dim3((unsigned)a.g.ntiles, p->B), dim3(NTHREADS),
                       p->lds[ax], p->stream, a);
  prof_stop(p, pk);
  HIPCHECK(hipGetLastError());
  return SFRDE_OK;
}

// The middle axis of a 3D field (y), in place on buffer B.
template <typename T>
int ypass(sfrde_plan_s* p, void* B) {
  if (p->ndim == 3) return launch_single<T>(p, 1, B, B, 0, 0);
  return SFRDE_OK;
}

// u_hat = F u and P = the partial inverse of cs*u_hat that the first X
// kernel expects (everything but the x axis).
template <typename T>
int prologue_physical(sfrde_plan_s* p, const void* state) {
  TRY(launch_single<T>(p, 0, state, p->P, 0, 0));
  TRY(ypass<T>(p, p->P));
  TRY(launch_z<T>(p, MODE_INIT, nullptr, nullptr));
  return ypass<T>(p, p->P);
}

// P from a stored spectral state (a checkpoint slot), read in place; the
// plan's u_hat is set from it when `set_uhat` (a forward continuation).
template <typename T>
int prologue_spectral(sfrde_plan_s* p, const void* spec, bool set_uhat = true) {
  if (set_uhat)
    HIPCHECK(hipMemcpyAsync(p->uhat, spec, field_bytes(p), hipMemcpyDeviceToDevice, p->stream));
  TRY(launch_z<T>(p, MODE_RESTORE, set_uhat ? p->uhat : spec, nullptr));
  return ypass<T>(p, p->P);
}

// One step of eq. ETDRK4P13 from t (four stages); stores stage data if asked.
// uh_in / uh_out: where the step reads u_hat and writes the next one (NULL:
// the plan's u_hat); the recompute of a segment reads and writes the
// segment store's slots, so that u_hat of every step is stored without a
// copy.
template <typename T>
int run_step(sfrde_plan_s* p, double t, const StepStore<T>* st, T* uh_in = nullptr,
             T* uh_out = nullptr) {
  const double off[4] = {0.0, 0.5 * p->dt, 0.5 * p->dt, p->dt};
  for (int j = 0; j < 4; ++j) {
    TRY(launch_x<T>(p, j, t + off[j], st ? st->phys : nullptr));
    TRY(ypass<T>(p, p->P));
    TRY(launch_z<T>(p, j, nullptr, st ? st->fhat : nullptr, j == 3 ? uh_out : uh_in));
    TRY(ypass<T>(p, p->P));
  }
  return SFRDE_OK;
}

template <typename T>
int fill(sfrde_plan_s* p, T* ptr, long long n, T v) {
  if (n <= 0) return SFRDE_OK;
  long long blocks = std::min<long long>((n + NTHREADS - 1) / NTHREADS, 65536);
  hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)blocks), dim3(NTHREADS), 0, p->stream, ptr, n, v);
  HIPCHECK(hipGetLastError());
  return SFRDE_OK;
}

// Checkpoint header words: magic, nsteps, K, S, total, dtype, ndim, bc, B,
// then the unknowns per axis n[0..2] (a transposed shape or another
// boundary condition has another spectral basis and must not be resumed).
CkptHeader header_words(const sfrde_plan_s* p, long long nsteps, long long K) {
  CkptHeader h{};
  const long long w[CKPT_WORDS] = {CKPT_MAGIC, nsteps, K, (long long)p->S, p->total,
                                   (long long)p->dtype, (long long)p->ndim, (long long)p->bc,
                                   (long long)p->B, p->n[0], p->n[1], p->n[2]};
  for (int i = 0; i < CKPT_WORDS; ++i) h.w[i] = w[i];
  return h;
}

int write_header(sfrde_plan_s* p, void* ckpt, long long nsteps, long long K) {
  hipLaunchKernelGGL(k_header, dim3(1), dim3(64), 0, p->stream, (long long*)ckpt,
                     header_words(p, nsteps, K));
  HIPCHECK(hipGetLastError());
  return SFRDE_OK;
}

// Reads the header of ckpt into h and checks that this plan wrote it (every
// word but nsteps and K).
int read_header(sfrde_plan_s* p, const void* ckpt, long long (&h)[CKPT_WORDS]) {
  HIPCHECK(hipMemcpyAsync(h, ckpt, sizeof(h), hipMemcpyDeviceToHost, p->stream));
  HIPCHECK(hipStreamSynchronize(p->stream));
  if (h[0] != CKPT_MAGIC) return fail(SFRDE_ESTATE, "checkpoint has no valid header");
  const CkptHeader mine = header_words(p, 0, 0);
  static const char* const what[CKPT_WORDS] = {"", "", "", "species count", "point count",
                                               "dtype", "dimension", "boundary condition",
                                               "ensemble size", "x size", "y size", "z size"};
  for (int i = 3; i < CKPT_WORDS; ++i)
    if (h[i] != mine.w[i])
      return fail(SFRDE_ESTATE, "checkpoint was written by a plan of another %s (%lld != %lld)",
                  what[i], h[i], mine.w[i]);
  if (h[2] < 1 || h[1] < 1) return fail(SFRDE_ESTATE, "checkpoint header has no steps");
  return SFRDE_OK;
}

int check_header(sfrde_plan_s* p, const void* ckpt, long long nsteps, long long K) {
  long long h[CKPT_WORDS];
  TRY(read_header(p, ckpt, h));
  if (h[2] != K) return fail(SFRDE_ESTATE, "checkpoint spacing %lld != %lld", h[2], K);
  if (h[1] < nsteps) return fail(SFRDE_ESTATE, "checkpoint covers %lld < %lld steps", h[1], nsteps);
  return SFRDE_OK;
}

char* ckpt_slot(sfrde_plan_s* p, void* ckpt, long long slot) {
  return (char*)ckpt + SFRDE_CKPT_HEADER_BYTES + (size_t)slot * field_bytes(p);
}

template <typename T>
int finish_forward(sfrde_plan_s* p, void* state) {
  TRY(launch_single<T>(p, 0, p->P, state, 0, 0));
  HIPCHECK(hipMemcpyAsync(p->h_flag, p->flag, sizeof(int), hipMemcpyDeviceToHost, p->stream));
  HIPCHECK(hipStreamSynchronize(p->stream));
  if (*p->h_flag) return fail(SFRDE_ENONFINITE, "a stage value or reaction became non-finite");
  return SFRDE_OK;
}

template <typename T>
int run_steps(sfrde_plan_s* p, long long k0, long long nsteps, double t0, long long K, void* ckpt) {
  for (long long k = 0; k < nsteps; ++k) {
    if (ckpt && K > 0 && k % K == 0)
      HIPCHECK(hipMemcpyAsync(ckpt_slot(p, ckpt, k / K), p->uhat, field_bytes(p),
                              hipMemcpyDeviceToDevice, p->stream));
    TRY(run_step<T>(p, t0 + double(k0 + k) * p->dt, (const StepStore<T>*)nullptr));
  }
  return SFRDE_OK;
}

template <typename T>
int integrate_t(sfrde_plan_s* p, void* state, long long nsteps, double t0, long long K, void* ckpt) {
  TRY(fill<int>(p, p->flag, 1, 0));
  if (ckpt && K > 0) TRY(write_header(p, ckpt, nsteps, K));
  TRY(prologue_physical<T>(p, state));
  TRY(run_steps<T>(p, 0, nsteps, t0, K, ckpt));
  return finish_forward<T>(p, state);
}

template <typename T>
int resume_t(sfrde_plan_s* p, const void* ckpt, long long slot, void* state, long long nsteps,
             double t0, long long K, void* ckpt_out) {
  TRY(fill<int>(p, p->flag, 1, 0));
  if (ckpt_out && K > 0) TRY(write_header(p, ckpt_out, nsteps, K));
  TRY(prologue_spectral<T>(p, ckpt_slot(p, (void*)ckpt, slot)));
  TRY(run_steps<T>(p, 0, nsteps, t0, K, ckpt_out));
  return finish_forward<T>(p, state);
}

// --------------------------------------------------------------------------
// The FP64 adjoint x kernel of reaction kind KIND (two species).
template <int KIND>
void launch_xadj64(sfrde_plan_s* p, dim3 grid, dim3 block, size_t lds,
                   const StageArgs<double>& a) {
  hipLaunchKernelGGL((k_xadj_m<double, XfX<double>, false, 2, false, KIND>), grid, block, lds,
                     p->stream, a, p->mfax[0]);
}

template <typename T>
int launch_xadj(sfrde_plan_s* p, int stage, const StepStore<T>& st) {
  StageArgs<T> a = stage_args<T>(p, 0, p->Pa);
  a.mode = stage;
  a.st_phys = st.phys;
  a.rp_acc = p->rp_acc;
  const long long pk = prof_start(p, KC_XADJ);
  if (p->use_m[0]) {
    const dim3 grid(p->grid_m[0], p->B), block(XfX<T>::THREADS);
    const bool fast = use_fast<T>(p, 0, {p->Pa});
    if constexpr (std::is_same<T, double>::value) {
      // FP64, two species: the instance of the plan's reaction kind
      if (p->S == 2 && p->rxn.kind <= RXN_GM) {
        const size_t lds = p->lds_m[0];
        switch (p->rxn.kind) {
          case RXN_LINEAR: launch_xadj64<RXN_LINEAR>(p, grid, block, lds, a); break;
          case RXN_FHN: launch_xadj64<RXN_FHN>(p, grid, block, lds, a); break;
          case RXN_GRAY_SCOTT: launch_xadj64<RXN_GRAY_SCOTT>(p, grid, block, lds, a); break;
          case RXN_SCHNAKENBERG: launch_xadj64<RXN_SCHNAKENBERG>(p, grid, block, lds, a); break;
          default: launch_xadj64<RXN_GM>(p, grid, block, lds, a); break;
        }
        goto xadj_launched;
      }
    }
    if (std::is_same<T, float>::value && fast && p->S == 1)
      hipLaunchKernelGGL((k_xadj_m<T, XfX<T>, true, 1>), grid, block, p->lds_m[0], p->stream, a,
                         p->mfax[0]);
    else if (std::is_same<T, float>::value && fast && p->S == 2 && p->mfax[0].direct &&
             !p->rp_acc)
      // DCT-I / DST-I, no reaction-parameter partials: the input folded
      // straight from registers
      hipLaunchKernelGGL((k_xadj_m<T, XfX<T>, true, 2, true>), grid, block, p->lds_m[0], p->stream,
                         a, p->mfax[0]);
    else if (std::is_same<T, float>::value && fast && p->S == 2)
      hipLaunchKernelGGL((k_xadj_m<T, XfX<T>, true, 2>), grid, block, p->lds_m[0], p->stream, a,
                         p->mfax[0]);
    else if (fast)
      hipLaunchKernelGGL((k_xadj_m<T, XfX<T>, std::is_same<T, float>::value>), grid, block,
                         p->lds_m[0], p->stream, a, p->mfax[0]);
    else
      hipLaunchKernelGGL((k_xadj_m<T, XfX<T>, false>), grid, block, p->lds_m[0], p->stream, a,
                         p->mfax[0]);
  xadj_launched:;
  } else if (p->use_f[0]) {
    hipLaunchKernelGGL((k_xadj<T, FftXf, true>), dim3((unsigned)a.g.ntiles, p->B), dim3(p->thr_f[0]),
                       p->lds_f[0], p->stream, a);
  } else
    hipLaunchKernelGGL(k_xadj<T>, dim3((unsigned)a.g.ntiles, p->B), dim3(NTHREADS),
                       p->lds[0], p->stream, a);
  prof_stop(p, pk);
  HIPCHECK(hipGetLastError());
  return SFRDE_OK;
}

template <typename T>
int launch_zadj(sfrde_plan_s* p, int mode, const StepStore<T>* st, int last) {
  const int ax = p->ndim - 1;
  StageArgs<T> a = stage_args<T>(p, ax, p->Pa);
  a.mode = mode;
  a.last = last;
  a.G = p->G;
  a.thp = p->thp_on ? p->thp : nullptr;
  if (st) {
    a.st_uhat = st->uhat;
    a.st_fhat = st->fhat;
  }
  if (!p->G) a.dcoef = nullptr;
  const long long pk = prof_start(p, KC_ZADJ);
  if (p->use_m[ax]) {
    const dim3 grid(p->grid_m[ax], p->B), block(XfZ<T>::THREADS);
    const size_t lds = p->lds_m[ax];
    const bool fast = use_fast<T>(p, ax, {p->Pa});
    // per-stage kernels: L formed in the kernel, no per-point accumulator
    const bool staged = fast && p->lfly && (p->thp_on || !p->G) && mode >= 0 && mode <= MODE_INIT;
    if constexpr (std::is_same<T, float>::value) {
      if (staged) {
        // the instance with or without the kappa/alpha partials
        const MfmaAxisDev& mx = p->mfax[ax];
        hipStream_t sm = p->stream;
        if (p->thp_on) {
          switch (mode) {
            case 0: hipLaunchKernelGGL((k_zadj_m<T, XfZ<T>, true, 0, 1>), grid, block, lds, sm, a, mx); break;
            case 1: hipLaunchKernelGGL((k_zadj_m<T, XfZ<T>, true, 1, 1>), grid, block, lds, sm, a, mx); break;
            case 2: hipLaunchKernelGGL((k_zadj_m<T, XfZ<T>, true, 2, 1>), grid, block, lds, sm, a, mx); break;
            case 3: hipLaunchKernelGGL((k_zadj_m<T, XfZ<T>, true, 3, 1>), grid, block, lds, sm, a, mx); break;
            default: hipLaunchKernelGGL((k_zadj_m<T, XfZ<T>, true, MODE_INIT, 1>), grid, block, lds, sm, a, mx); break;
          }
        } else {
          switch (mode) {
            case 0: hipLaunchKernelGGL((k_zadj_m<T, XfZ<T>, true, 0, 0>), grid, block, lds, sm, a, mx); break;
            case 1: hipLaunchKernelGGL((k_zadj_m<T, XfZ<T>, true, 1, 0>), grid, block, lds, sm, a, mx); break;
            case 2: hipLaunchKernelGGL((k_zadj_m<T, XfZ<T>, true, 2, 0>), grid, block, lds, sm, a, mx); break;
            case 3: hipLaunchKernelGGL((k_zadj_m<T, XfZ<T>, true, 3, 0>), grid, block, lds, sm, a, mx); break;
            default: hipLaunchKernelGGL((k_zadj_m<T, XfZ<T>, true, MODE_INIT, 0>), grid, block, lds, sm, a, mx); break;
          }
        }
        goto zadj_launched;
      }
    }
    if (fast)
      hipLaunchKernelGGL((k_zadj_m<T, XfZ<T>, std::is_same<T, float>::value>), grid, block,
                         p->lds_m[ax], p->stream, a, p->mfax[ax]);
    else
      hipLaunchKernelGGL((k_zadj_m<T, XfZ<T>, false>), grid, block, p->lds_m[ax], p->stream, a,
                         p->mfax[ax]);
  } else if (p->use_f[ax]) {
    hipLaunchKernelGGL((k_zadj<T, FftXf, true>), dim3((unsigned)a.g.ntiles, p->B), dim3(p->thr_f[ax]),
                       p->lds_f[ax], p->stream, a);
  } else
    hipLaunchKernelGGL(k_zadj<T>, dim3((unsigned)a.g.ntiles, p->B), dim3(NTHREADS),
                       p->lds[ax], p->stream, a);
zadj_launched:
  prof_stop(p, pk);
  HIPCHECK(hipGetLastError());
  return SFRDE_OK;
}

// Reverse sweep over one step whose stage data sit in `st`.
template <typename T>
int adjoint_step(sfrde_plan_s* p, const StepStore<T>& st, int last) {
  // adjoint stage m visits the forward stage value 3 - m (c, b, a, u)
  for (int m = 0; m < 4; ++m) {
    TRY(launch_xadj<T>(p, 3 - m, st));
    TRY(ypass<T>(p, p->Pa));
    TRY(launch_zadj<T>(p, m, &st, last));
    TRY(ypass<T>(p, p->Pa));
  }
  return SFRDE_OK;
}

// Coefficient arguments of member b (eigenvalue tables, kappa, alpha).
CoefArgs coef_args(const sfrde_plan_s* p, int b, int deriv) {
  CoefArgs c{};
  c.lam0 = p->lam[0];
  c.lam1 = p->lam[1];
  c.lam2 = p->lam[2] ? p->lam[2] : p->lam[1];
  c.n0 = p->n[0];
  c.n1 = p->n[1];
  c.n2 = p->n[2];
  c.total = p->total;
  c.S = p->S;
  c.scheme = p->scheme;
  c.deriv = deriv;
  c.tau = p->dt;
  for (int s = 0; s < p->S; ++s) {
    c.alpha[s] = p->alpha_m[(size_t)b * p->S + s];
    c.kappa[s] = p->kappa_m[(size_t)b * p->S + s];
  }
  return c;
}

// Per-point tables of every member, [B][k][S][total]: deriv 0 the six
// coefficients (k = 6), 1 their d/dL (k = 6), 2 L itself (k = 1).
int coef_tables(sfrde_plan_s* p, int deriv, void* out) {
  const size_t per = (size_t)(deriv == 2 ? 1 : NCOEF) * p->S * p->total;
  const long long blocks = std::min<long long>((p->total + NTHREADS - 1) / NTHREADS, 8192);
  for (int b = 0; b < p->B; ++b) {
    const CoefArgs c = coef_args(p, b, deriv);
    if (p->dtype == SFRDE_F32)
      hipLaunchKernelGGL(k_coefs<float>, dim3((unsigned)blocks), dim3(NTHREADS), 0, p->stream, c,
                         (float*)out + b * per);
    else
      hipLaunchKernelGGL(k_coefs<double>, dim3((unsigned)blocks), dim3(NTHREADS), 0, p->stream,
                         c, (double*)out + b * per);
    HIPCHECK(hipGetLastError());
  }
  return SFRDE_OK;
}

// Blocks of the adjoint X kernel (each owns one accumulator per parameter).
long long rp_blocks(const sfrde_plan_s* p) {
  return p->use_m[0] ? (long long)p->grid_m[0]
                      : p->use_f[0] ? p->geom_f[0].ntiles : p->geom[0].ntiles;
}

// Bytes of the backward buffers (what ensure_backward_buffers allocates),
// each rounded up to 256 bytes as carve_backward_buffers lays them out.
size_t round256(size_t b) { return (b + 255) / 256 * 256; }

// The backward buffers laid out in the static scratch array (no allocation;
// the plan's own pointers are saved and restored by the caller). Fails with
// EINVAL, before any device work, if they do not fit.
int carve_backward_buffers(sfrde_plan_s* p, long long seg_steps, bool want_theta, bool want_p) {
  const size_t f = field_bytes(p);
  char* base = static_cast<char*>(p->scratch);
  size_t off = 0;
  auto take = [&](void** ptr, size_t bytes) {
    *ptr = base + off;
    off += round256(bytes);
  };
  take(&p->Pa, f);
  take(&p->zh, f);
  take(&p->aacc, f);
  take(&p->ahat, f);
  take(&p->gu, f);
  take(&p->seg, (size_t)seg_steps * p->seg_stride * f);
  p->seg_steps = seg_steps;
  p->seg_cap = seg_steps * p->seg_stride;
  p->thp = nullptr;
  p->G = nullptr;
  p->dcoef = nullptr;
  p->rp_acc = nullptr;
  bool fill_dcoef = false;
  if (want_theta && p->thp_on) {
    take((void**)&p->thp, (size_t)4 * p->grid_m[p->ndim - 1] * sizeof(double));
  } else if (want_theta) {
    take((void**)&p->G, field_elems(p) * sizeof(double));
    // FP64 P13 plans form the coefficient derivatives from L in the combine
    if (!(p->ltab && p->dtype == SFRDE_F64)) {
      take(&p->dcoef, NCOEF * f);
      fill_dcoef = true;
    }
  }
  if (want_p) take((void**)&p->rp_acc, (size_t)p->B * MAX_PARAMS * rp_blocks(p) * sizeof(double));
  const long long need = RED_OUT + (long long)p->B * RED_PER_MEMBER;
  take((void**)&p->red, (size_t)need * sizeof(double));
  p->red_len = need;
  if (off > SCRATCH_BYTES)
    return fail(SFRDE_EINVAL,
                "this backward needs %zu bytes of workspace; the allocation-free entry point "
                "holds %zu (use sfrde_backward, or a smaller ckpt_every or grid)",
                off, SCRATCH_BYTES);
  if (fill_dcoef) TRY(coef_tables(p, 1, p->dcoef));
  return SFRDE_OK;
}

int ensure_backward_buffers(sfrde_plan_s* p, long long seg_steps, bool want_theta, bool want_p) {
  if (p->noalloc) return carve_backward_buffers(p, seg_steps, want_theta, want_p);
  const size_t f = field_bytes(p);
  TRY(dev_alloc(p, &p->Pa, f));
  TRY(dev_alloc(p, &p->zh, f));
  TRY(dev_alloc(p, &p->aacc, f));
  TRY(dev_alloc(p, &p->ahat, f));
  TRY(dev_alloc(p, &p->gu, f));
  const long long seg_need = seg_steps * p->seg_stride;
  if (p->seg && p->seg_cap < seg_need) {
    dev_free(p, &p->seg, (size_t)p->seg_cap * f);
    p->seg_cap = 0;
  }
  if (!p->seg) {
    TRY(dev_alloc(p, &p->seg, (size_t)seg_need * f));
    p->seg_cap = seg_need;
  }
  p->seg_steps = seg_steps;
  if (want_theta && p->thp_on) {
    TRY(dev_alloc(p, (void**)&p->thp, (size_t)4 * p->grid_m[p->ndim - 1] * sizeof(double)));
  } else if (want_theta) {
    TRY(dev_alloc(p, (void**)&p->G, field_elems(p) * sizeof(double)));
    // FP64 P13 plans form the coefficient derivatives from L in the combine
    if (!p->dcoef && !(p->ltab && p->dtype == SFRDE_F64)) {
      TRY(dev_alloc(p, &p->dcoef, NCOEF * f));
      TRY(coef_tables(p, 1, p->dcoef));
    }
  }
  if (want_p) {
    TRY(dev_alloc(p, (void**)&p->rp_acc,
                  (size_t)p->B * MAX_PARAMS * rp_blocks(p) * sizeof(double)));
  }
  const long long need = RED_OUT + (long long)p->B * RED_PER_MEMBER;
  if (p->red && p->red_len < need) dev_free(p, (void**)&p->red, p->red_len * sizeof(double));
  if (!p->red) {
    TRY(dev_alloc(p, (void**)&p->red, need * sizeof(double)));
    p->red_len = need;
  }
  return SFRDE_OK;
}

template <typename T>
int backward_t(sfrde_plan_s* p, const void* ckpt, long long nsteps, long long K, double t0,
               const void* grad_uT, void* grad_u0, double* gk, double* ga, double* gp) {
  const bool want_theta = gk || ga;
  const bool want_p = gp != nullptr && p->rxn.np > 0;
  const long long seg_steps = std::min(K, nsteps);
  // the recompute stores the stage values; u_hat and the four f_hat only for
  // the kappa/alpha terms
  p->seg_stride = want_theta ? 9 : 4;
  // kappa/alpha gradients formed inside the vector adjoint Z kernels (L
  // formed there too), else through the per-point accumulator G
  p->thp_on = want_theta && p->lfly && p->B == 1 && p->S <= 2 && use_fast<T>(p, p->ndim - 1, {});
  {
    const int rc0 = ensure_backward_buffers(p, seg_steps, want_theta, want_p);
    if (rc0 != SFRDE_OK) {
      p->thp_on = false;
      return rc0;
    }
  }
  // Buffers from an earlier call stay allocated; accumulate only what is asked.
  double* G_saved = p->G;
  if (!want_theta || p->thp_on) p->G = nullptr;
  if (p->G) TRY(fill<double>(p, p->G, (long long)field_elems(p), 0.0));
  const long long zgrid = p->grid_m[p->ndim - 1];
  if (p->thp_on) TRY(fill<double>(p, p->thp, 4 * zgrid, 0.0));
  double* rp_saved = p->rp_acc;
  if (!want_p) p->rp_acc = nullptr;
  if (p->rp_acc)
    TRY(fill<double>(p, p->rp_acc, (long long)p->B * MAX_PARAMS * rp_blocks(p), 0.0));

  int rc = SFRDE_OK;
  do {
    // cotangent of u(T) into the adjoint variables, then its first stage input
    if ((rc = launch_single<T>(p, 0, grad_uT, p->Pa, 1, 0))) break;
    if ((rc = ypass<T>(p, p->Pa))) break;
    if ((rc = launch_zadj<T>(p, MODE_INIT, nullptr, 0))) break;
    if ((rc = ypass<T>(p, p->Pa))) break;
    const long long nseg = (nsteps + K - 1) / K;
    for (long long sgi = nseg - 1; sgi >= 0 && rc == SFRDE_OK; --sgi) {
      const long long k0 = sgi * K, k1 = std::min(nsteps, k0 + K);
      // the segment's u_hat of step k sits in store slot k - k0, that of its
      // first step in the checkpoint itself (read in place)
      // (without the kappa/alpha terms u_hat is not stored: the recompute
      // runs on the plan's own)
      T* ck = reinterpret_cast<T*>(ckpt_slot(p, (void*)ckpt, sgi));
      const bool keep_uhat = p->seg_stride == 9;
      auto store_at = [&](long long k) {
        StepStore<T> st = step_store<T>(p, k - k0);
        if (k == k0 && keep_uhat) st.uhat = ck;
        return st;
      };
      if ((rc = prologue_spectral<T>(p, ck, !keep_uhat))) break;
      for (long long k = k0; k < k1 && rc == SFRDE_OK; ++k) {
        StepStore<T> st = store_at(k);
        T* out = k + 1 < k1 ? store_at(k + 1).uhat : (T*)p->uhat;
        rc = run_step<T>(p, t0 + double(k) * p->dt, &st, st.uhat, keep_uhat ? out : nullptr);
      }
      for (long long k = k1 - 1; k >= k0 && rc == SFRDE_OK; --k) {
        StepStore<T> st = store_at(k);
        rc = adjoint_step<T>(p, st, k == 0);
      }
    }
    if (rc) break;
    if (grad_u0 && (rc = launch_single<T>(p, 0, p->Pa, grad_u0, 0, 1))) break;
    const int nb = 1024;
    double* rout = p->red + RED_OUT;
    for (int m = 0; m < p->B && rc == SFRDE_OK; ++m) {
      double* ro = rout + (size_t)m * RED_PER_MEMBER;
      if (want_theta && p->thp_on) {  // one member only (L formed in the kernels)
        hipLaunchKernelGGL(k_rowsum, dim3(2 * p->S), dim3(NTHREADS), 0, p->stream, p->thp, zgrid,
                           ro);
        if (hipGetLastError() != hipSuccess) { rc = fail(SFRDE_EDEVICE, "k_rowsum launch"); break; }
      } else if (want_theta) {
        const CoefArgs c = coef_args(p, m, 0);
        hipLaunchKernelGGL(k_greduce, dim3(nb), dim3(NTHREADS), 0, p->stream, c,
                           p->G + (size_t)m * p->S * p->total, p->cs,
                           (int)(p->bc == SFRDE_BC_NEUMANN), p->red);
        if (hipGetLastError() != hipSuccess) { rc = fail(SFRDE_EDEVICE, "k_greduce launch"); break; }
        hipLaunchKernelGGL(k_rowsum, dim3(2 * p->S), dim3(NTHREADS), 0, p->stream, p->red,
                           (long long)nb, ro);
        if (hipGetLastError() != hipSuccess) { rc = fail(SFRDE_EDEVICE, "k_rowsum launch"); break; }
      }
      if (want_p) {
        hipLaunchKernelGGL(k_rowsum, dim3(p->rxn.np), dim3(NTHREADS), 0, p->stream,
                           p->rp_acc + (size_t)m * MAX_PARAMS * rp_blocks(p), rp_blocks(p),
                           ro + 2 * MAX_SPECIES);
        if (hipGetLastError() != hipSuccess) { rc = fail(SFRDE_EDEVICE, "k_rowsum launch"); break; }
      }
    }
    if (rc) break;
    if (hipStreamSynchronize(p->stream) != hipSuccess) {
      rc = fail(SFRDE_EDEVICE, "stream synchronize");
      break;
    }
    // the members' sums, copied in chunks through a buffer on the stack
    constexpr int CHUNK = 64;
    double host[CHUNK * RED_PER_MEMBER];
    for (int m0 = 0; m0 < p->B && (want_theta || want_p); m0 += CHUNK) {
      const int nm = std::min(CHUNK, p->B - m0);
      if (hipMemcpyAsync(host, rout + (size_t)m0 * RED_PER_MEMBER,
                         (size_t)nm * RED_PER_MEMBER * sizeof(double), hipMemcpyDeviceToHost,
                         p->stream) != hipSuccess ||
          hipStreamSynchronize(p->stream) != hipSuccess) {
        rc = fail(SFRDE_EDEVICE, "copy of gradient partials");
        break;
      }
      for (int i = 0; i < nm; ++i) {
        const int m = m0 + i;
        const double* hm = host + (size_t)i * RED_PER_MEMBER;
        for (int s = 0; s < p->S; ++s) {
          if (gk) gk[m * p->S + s] = hm[2 * s];
          if (ga) ga[m * p->S + s] = hm[2 * s + 1];
        }
        if (want_p)
          for (int k = 0; k < p->rxn.np; ++k) gp[m * p->rxn.np + k] = hm[2 * MAX_SPECIES + k];
      }
    }
  } while (0);
  p->G = G_saved;
  p->rp_acc = rp_saved;
  p->thp_on = false;
  return rc;
}

void destroy_plan(sfrde_plan_s* p) {
  if (!p) return;
  (void)hipStreamSynchronize(p->stream);
  void** ptrs[] = {&p->Mt[0], &p->Mt[1], &p->Mt[2], (void**)&p->lam[0], (void**)&p->lam[1],
                   (void**)&p->lam[2], &p->coef, &p->dcoef, &p->ltab, &p->P, &p->uhat, &p->ctil, &p->acc,
                   &p->Pa, &p->zh, &p->aacc, &p->ahat, &p->gu, (void**)&p->G, &p->seg,
                   (void**)&p->rp_acc, (void**)&p->thp, (void**)&p->red, (void**)&p->flag, (void**)&p->rxm, &p->tw[0], &p->tw[1], &p->tw[2], &p->mf_A[0],
                   &p->mf_A[1], &p->mf_A[2]};
  for (void** q : ptrs) {
    if (*q) (void)hipFree(*q);
    *q = nullptr;
  }
  if (p->h_flag) (void)hipHostFree(p->h_flag);
  for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
  delete p;
}

int validate(int32_t ndim, const int64_t* n, int32_t bc, const double* h, int32_t S,
             const double* alpha, const double* kappa, double dt, int32_t reaction,
             int32_t nparams, const double* params, int32_t dtype, int32_t scheme) {
  if (ndim < 1 || ndim > 3) return fail(SFRDE_EINVAL, "ndim must be 1, 2 or 3 (got %d)", ndim);
  if (!n || !h) return fail(SFRDE_EINVAL, "n and h must not be NULL");
  for (int a = 0; a < ndim; ++a) {
    if (n[a] < 2 || n[a] > MAX_N)
      return fail(SFRDE_EINVAL, "n[%d] = %lld outside [2, %d]", a, (long long)n[a], MAX_N);
    if (!(h[a] > 0.0) || !std::isfinite(h[a]))
      return fail(SFRDE_EINVAL, "h[%d] must be finite and > 0", a);
  }
  if (bc < 0 || bc > 2) return fail(SFRDE_EINVAL, "unknown boundary condition %d", bc);
  if (S < 1 || S > MAX_SPECIES) return fail(SFRDE_EINVAL, "nspecies %d outside [1, 4]", S);
  if (!alpha || !kappa) return fail(SFRDE_EINVAL, "alpha and kappa must not be NULL");
  for (int s = 0; s < S; ++s) {
    if (!(alpha[s] > 0.0 && alpha[s] <= 2.0))
      return fail(SFRDE_EINVAL, "alpha[%d] = %g outside (0, 2]", s, alpha[s]);
    if (!(kappa[s] >= 0.0) || !std::isfinite(kappa[s]))
      return fail(SFRDE_EINVAL, "kappa[%d] must be finite and >= 0", s);
  }
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(SFRDE_EINVAL, "dt must be finite and > 0");
  if (reaction < 0 || reaction > RXN_FISHER_MMS)
    return fail(SFRDE_EINVAL, "unknown reaction %d", reaction);
  if (reaction >= RXN_HUXLEY_MMS) {
    if (S != 1) return fail(SFRDE_EINVAL, "reaction %d needs exactly 1 species", reaction);
    if (reaction == RXN_HUXLEY_MMS && (ndim != 2 || bc == SFRDE_BC_DIRICHLET))
      return fail(SFRDE_EINVAL, "the Example 2 source is for 2D periodic or Neumann grids");
    if (reaction == RXN_FISHER_MMS && (ndim != 1 || bc != SFRDE_BC_DIRICHLET))
      return fail(SFRDE_EINVAL, "the Example 1 source is for 1D Dirichlet grids");
  } else if (reaction != RXN_LINEAR && S != 2) {
    return fail(SFRDE_EINVAL, "reaction %d needs exactly 2 species", reaction);
  }
  if (nparams != expected_nparams(reaction, S))
    return fail(SFRDE_EINVAL, "reaction %d takes %d parameters (got %d)", reaction,
                expected_nparams(reaction, S), nparams);
  if (nparams > 0 && !params) return fail(SFRDE_EINVAL, "params must not be NULL");
  for (int k = 0; k < nparams; ++k)
    if (!std::isfinite(params[k])) return fail(SFRDE_EINVAL, "params[%d] is not finite", k);
  if (dtype != SFRDE_F32 && dtype != SFRDE_F64) return fail(SFRDE_EINVAL, "unknown dtype %d", dtype);
  if (scheme != SFRDE_SCHEME_P13 && scheme != SFRDE_SCHEME_EXP)
    return fail(SFRDE_EINVAL, "unknown scheme %d", scheme);
  return SFRDE_OK;
}

template <typename T>
int upload_matrix(sfrde_plan_s* p, int axis) {
  const long long n = p->n[axis];
  std::vector<double> Mt = axis_matrix_t(p->bc, n);
  std::vector<T> conv(Mt.size());
  for (size_t i = 0; i < Mt.size(); ++i) conv[i] = T(Mt[i]);
  TRY(dev_alloc(p, &p->Mt[axis], conv.size() * sizeof(T)));
  HIPCHECK(hipMemcpy(p->Mt[axis], conv.data(), conv.size() * sizeof(T), hipMemcpyHostToDevice));
  return SFRDE_OK;
}

int build_plan(sfrde_plan_s* p) {
  int dev = 0;
  HIPCHECK(hipGetDevice(&dev));
  HIPCHECK(hipDeviceGetAttribute(&p->n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  p->device = dev;
  TRY(scratch_address(dev, &p->scratch));
  for (int a = 0; a < p->ndim; ++a) {
    std::vector<double> lam(p->n[a]);
    for (long long k = 0; k < p->n[a]; ++k)
      lam[k] = p->n[a] == 1 ? 0.0 : axis_eigenvalue(p->bc, p->n[a], p->h[a], k);
    TRY(dev_alloc(p, (void**)&p->lam[a], lam.size() * sizeof(double)));
    HIPCHECK(hipMemcpy(p->lam[a], lam.data(), lam.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  size_t lds_max = 0;
  // dense tiles narrowed until the launch (all members) fills the device
  for (int a = 0; a < p->ndim; ++a)
    make_geom(p, a, std::max<long long>(1, (2LL * p->n_cu + p->B - 1) / p->B));
  for (int a = 0; a < p->ndim; ++a) TRY(setup_mfma_axis(p, a));
  // Long periodic axes of 256, 512 or 1024 points: FFT kernels. Any other
  // axis the matrix-core engine does not take (n > 256, other periodic
  // n >= 256, the one-point padding axis of 1D plans) runs the dense LDS
  // kernels with the axis matrix.
  for (int a = 0; a < p->ndim; ++a) {
    if (p->dtype == SFRDE_F32)
      TRY(setup_fft_axis<float>(p, a));
    else
      TRY(setup_fft_axis<double>(p, a));
    if (!p->use_m[a] && !p->use_f[a]) {
      if (p->dtype == SFRDE_F32)
        TRY(upload_matrix<float>(p, a));
      else
        TRY(upload_matrix<double>(p, a));
    }
  }
  {
    // FP32 P13 plans whose last axis runs the vector Z kernels form L there
    // from the eigenvalue tables (kept in LDS as floats) instead of reading
    // an L table.
    const int za = p->ndim - 1;
    long long nsum = 0;
    for (int a = 0; a < p->ndim; ++a) nsum += p->n[a];
    const size_t extra = (size_t)nsum * sizeof(float);
    if (p->dtype == SFRDE_F32 && p->scheme == SFRDE_SCHEME_P13 && p->B == 1 &&
        p->use_m[za] &&
        p->geom_m[za].fast && p->n[0] % 4 == 0 && p->lds_m[za] + extra <= 160 * 1024) {
      p->lfly = true;
      p->lam_off = (p->lds_m[za] + 15) / 16 * 16;
      p->lds_m[za] = p->lam_off + extra;
    }
  }
  for (int a = 0; a < p->ndim; ++a) lds_max = std::max(lds_max, p->lds_m[a]);
  if (lds_max > 0) {
    if (p->dtype == SFRDE_F32)
      TRY(set_lds_attrs<float>(lds_max));
    else
      TRY(set_lds_attrs<double>(lds_max));
  }
  const size_t f = field_bytes(p);
  TRY(dev_alloc(p, &p->coef, NCOEF * f));
  TRY(dev_alloc(p, &p->P, f));
  TRY(dev_alloc(p, &p->uhat, f));
  TRY(dev_alloc(p, &p->ctil, f));
  TRY(dev_alloc(p, &p->acc, f));
  TRY(dev_alloc(p, (void**)&p->flag, 64));
  HIPCHECK(hipHostMalloc((void**)&p->h_flag, sizeof(int), hipHostMallocDefault));
  *p->h_flag = 0;
  if (p->B > 1) {
    TRY(dev_alloc(p, (void**)&p->rxm, p->rxn_m.size() * sizeof(Rxn)));
    HIPCHECK(hipMemcpy(p->rxm, p->rxn_m.data(), p->rxn_m.size() * sizeof(Rxn),
                       hipMemcpyHostToDevice));
  }
  TRY(coef_tables(p, 0, p->coef));
  if (p->scheme == SFRDE_SCHEME_P13) {
    // The forward combine forms the P13 coefficients from L: one table read
    // per species and stage instead of up to four. The six tables stay for
    // the adjoint.
    TRY(dev_alloc(p, &p->ltab, f));
    TRY(coef_tables(p, 2, p->ltab));
  }
  TRY(fill<int>(p, p->flag, 16, 0));
  HIPCHECK(hipStreamSynchronize(p->stream));
  return SFRDE_OK;
}

}  // namespace

// ==========================================================================
extern "C" {

const char* sfrde_last_error(void) { return g_err.c_str(); }

int sfrde_plan_batch(sfrde_plan_t* out, int32_t batch, int32_t ndim, const int64_t* n,
                     int32_t bc, const double* h, int32_t nspecies, const double* alpha,
                     const double* kappa, double dt, int32_t reaction, int32_t nparams,
                     const double* params, int32_t dtype, int32_t scheme, void* hip_stream) {
  g_err.clear();
  if (!out) return fail(SFRDE_EINVAL, "out must not be NULL");
  *out = nullptr;
  if (batch < 1 || batch > MAX_BATCH)
    return fail(SFRDE_EINVAL, "batch %d outside [1, %d]", batch, MAX_BATCH);
  if (!alpha || !kappa) return fail(SFRDE_EINVAL, "alpha and kappa must not be NULL");
  if (nparams > 0 && !params) return fail(SFRDE_EINVAL, "params must not be NULL");
  for (int b = 0; b < batch; ++b) {
    const int rc = validate(ndim, n, bc, h, nspecies, alpha + (size_t)b * nspecies,
                            kappa + (size_t)b * nspecies, dt, reaction, nparams,
                            params ? params + (size_t)b * nparams : nullptr, dtype, scheme);
    if (rc != SFRDE_OK) {
      if (batch > 1) g_err += " (ensemble member " + std::to_string(b) + ")";
      return rc;
    }
  }
  sfrde_plan_s* p = new (std::nothrow) sfrde_plan_s();
  if (!p) return fail(SFRDE_ENOMEM, "host allocation of the plan failed");
  // A 1D plan runs as a 2D one whose second axis has one point (eigenvalue
  // 0, identity transform, weight 1): the field layout is the same.
  p->ndim = ndim == 1 ? 2 : ndim;
  p->n[1] = 1;
  p->h[1] = 1.0;
  for (int a = 0; a < ndim; ++a) {
    p->n[a] = n[a];
    p->h[a] = h[a];
  }
  p->total = 1;
  for (int a = 0; a < p->ndim; ++a) {
    p->total *= p->n[a];
    p->cs *= axis_inverse_scale(bc, p->n[a]);
  }
  p->bc = bc;
  p->S = nspecies;
  p->B = batch;
  p->alpha_m.assign(alpha, alpha + (size_t)batch * nspecies);
  p->kappa_m.assign(kappa, kappa + (size_t)batch * nspecies);
  for (int s = 0; s < nspecies; ++s) {
    p->alpha[s] = alpha[s];
    p->kappa[s] = kappa[s];
  }
  p->dt = dt;
  p->rxn_m.resize(batch);
  for (int b = 0; b < batch; ++b) {
    Rxn& r = p->rxn_m[b];
    r = Rxn{};
    r.kind = reaction;
    r.S = nspecies;
    r.np = nparams;
    for (int k = 0; k < nparams; ++k) r.p[k] = params[(size_t)b * nparams + k];
    if (reaction >= RXN_HUXLEY_MMS) {
      // source constants of Examples 1 and 2 (Section 5.1), see mms_source()
      const double pi = 3.14159265358979323846, a = alpha[(size_t)b * nspecies],
                   k = kappa[(size_t)b * nspecies];
      double* c = r.p + MMS_P0;
      c[0] = a;
      if (reaction == RXN_HUXLEY_MMS) {
        c[1] = k / 16.0 * 9.0 * pow(8.0 * pi * pi, 0.5 * a);
        c[2] = k / 16.0 * 3.0 * pow(40.0 * pi * pi, 0.5 * a);
        c[3] = k / 16.0 * pow(72.0 * pi * pi, 0.5 * a);
      } else {
        c[1] = k / 4.0 * 3.0 * pow(2.0 * pi, a);
        c[2] = 0.0;
        c[3] = k / 4.0 * pow(6.0 * pi, a);
      }
      c[4] = h[0];
      c[5] = ndim > 1 ? h[1] : 0.0;
    }
  }
  p->rxn = p->rxn_m[0];
  p->dtype = dtype;
  p->scheme = scheme;
  p->stream = (hipStream_t)hip_stream;
  p->w = dtype == SFRDE_F32 ? 4 : 8;
  for (int a = 0; a < p->ndim; ++a) make_geom(p, a);
  int rc = build_plan(p);
  if (rc != SFRDE_OK) {
    std::string msg = g_err;
    destroy_plan(p);
    g_err = msg;
    return rc;
  }
  *out = p;
  return SFRDE_OK;
}

int sfrde_plan(sfrde_plan_t* out, int32_t ndim, const int64_t* n, int32_t bc, const double* h,
               int32_t nspecies, const double* alpha, const double* kappa, double dt,
               int32_t reaction, int32_t nparams, const double* params, int32_t dtype,
               int32_t scheme, void* hip_stream) {
  return sfrde_plan_batch(out, 1, ndim, n, bc, h, nspecies, alpha, kappa, dt, reaction, nparams,
                          params, dtype, scheme, hip_stream);
}

int sfrde_destroy(sfrde_plan_t plan) {
  g_err.clear();
  if (!plan) return fail(SFRDE_EINVAL, "plan is NULL");
  destroy_plan(plan);
  return SFRDE_OK;
}

int sfrde_integrate(sfrde_plan_t p, void* state, int64_t nsteps, double t0, int64_t ckpt_every,
                    void* ckpt) {
  g_err.clear();
  if (!p) return fail(SFRDE_EINVAL, "plan is NULL");
  if (!state) return fail(SFRDE_EINVAL, "state must not be NULL");
  if (nsteps < 0) return fail(SFRDE_EINVAL, "nsteps must be >= 0");
  if (ckpt_every < 0) return fail(SFRDE_EINVAL, "ckpt_every must be >= 0");
  if (!std::isfinite(t0)) return fail(SFRDE_EINVAL, "t0 must be finite");
  if (nsteps == 0) return SFRDE_OK;
  if (p->dtype == SFRDE_F32) return integrate_t<float>(p, state, nsteps, t0, ckpt_every, ckpt);
  return integrate_t<double>(p, state, nsteps, t0, ckpt_every, ckpt);
}

int sfrde_step(sfrde_plan_t p, void* state, double t) {
  return sfrde_integrate(p, state, 1, t, 0, nullptr);
}

int64_t sfrde_ckpt_bytes(sfrde_plan_t p, int64_t nsteps, int64_t ckpt_every) {
  g_err.clear();
  if (!p) return fail(SFRDE_EINVAL, "plan is NULL");
  if (nsteps < 1 || ckpt_every < 1)
    return fail(SFRDE_EINVAL, "nsteps and ckpt_every must be >= 1");
  const int64_t nslots = (nsteps + ckpt_every - 1) / ckpt_every;
  return SFRDE_CKPT_HEADER_BYTES + nslots * (int64_t)field_bytes(p);
}

int sfrde_resume(sfrde_plan_t p, const void* ckpt, int64_t slot, void* state, int64_t nsteps,
                 double t0, int64_t ckpt_every, void* ckpt_out) {
  g_err.clear();
  if (!p) return fail(SFRDE_EINVAL, "plan is NULL");
  if (!ckpt || !state) return fail(SFRDE_EINVAL, "ckpt and state must not be NULL");
  if (slot < 0 || nsteps < 0 || ckpt_every < 0) return fail(SFRDE_EINVAL, "negative argument");
  long long h[CKPT_WORDS];
  TRY(read_header(p, ckpt, h));
  const long long nslots = (h[1] + h[2] - 1) / h[2];
  if (slot >= nslots) return fail(SFRDE_ESTATE, "slot %lld >= %lld slots", (long long)slot, nslots);
  if (nsteps == 0) return SFRDE_OK;
  if (p->dtype == SFRDE_F32)
    return resume_t<float>(p, ckpt, slot, state, nsteps, t0, ckpt_every, ckpt_out);
  return resume_t<double>(p, ckpt, slot, state, nsteps, t0, ckpt_every, ckpt_out);
}

int sfrde_backward(sfrde_plan_t p, const void* ckpt, int64_t nsteps, int64_t ckpt_every,
                   double t0, const void* grad_uT, void* grad_u0, double* grad_kappa,
                   double* grad_alpha, double* grad_params) {
  g_err.clear();
  if (!p) return fail(SFRDE_EINVAL, "plan is NULL");
  if (!ckpt || !grad_uT) return fail(SFRDE_EINVAL, "ckpt and grad_uT must not be NULL");
  if (nsteps < 1 || ckpt_every < 1) return fail(SFRDE_EINVAL, "nsteps, ckpt_every must be >= 1");
  TRY(check_header(p, ckpt, nsteps, ckpt_every));
  if (p->rxn.kind >= RXN_HUXLEY_MMS && (grad_kappa || grad_alpha))
    return fail(SFRDE_EUNSUPPORTED,
                "kappa and alpha gradients of the manufactured sources are not implemented");
  if (p->dtype == SFRDE_F32)
    return backward_t<float>(p, ckpt, nsteps, ckpt_every, t0, grad_uT, grad_u0, grad_kappa,
                             grad_alpha, grad_params);
  return backward_t<double>(p, ckpt, nsteps, ckpt_every, t0, grad_uT, grad_u0, grad_kappa,
                            grad_alpha, grad_params);
}

int sfrde_backward_noalloc(sfrde_plan_t p, const void* ckpt, int64_t nsteps,
                           int64_t ckpt_every, double t0, const void* grad_uT, void* grad_u0,
                           double* grad_kappa, double* grad_alpha, double* grad_params) {
  g_err.clear();
  if (!p) return fail(SFRDE_EINVAL, "plan is NULL");
  if (!ckpt || !grad_uT) return fail(SFRDE_EINVAL, "ckpt and grad_uT must not be NULL");
  if (nsteps < 1 || ckpt_every < 1) return fail(SFRDE_EINVAL, "nsteps, ckpt_every must be >= 1");
  if (!p->scratch) return fail(SFRDE_EDEVICE, "the plan has no scratch address");
  TRY(check_header(p, ckpt, nsteps, ckpt_every));
  if (p->rxn.kind >= RXN_HUXLEY_MMS && (grad_kappa || grad_alpha))
    return fail(SFRDE_EUNSUPPORTED,
                "kappa and alpha gradients of the manufactured sources are not implemented");
  // the plan's own backward buffers are set aside for this call
  void* saved[] = {p->Pa, p->zh, p->aacc, p->ahat, p->gu, p->seg, p->G, p->dcoef, p->rp_acc,
                   p->thp, p->red};
  const long long saved_seg = p->seg_steps, saved_red = p->red_len, saved_cap = p->seg_cap;
  p->noalloc = true;
  int rc;
  if (p->dtype == SFRDE_F32)
    rc = backward_t<float>(p, ckpt, nsteps, ckpt_every, t0, grad_uT, grad_u0, grad_kappa,
                           grad_alpha, grad_params);
  else
    rc = backward_t<double>(p, ckpt, nsteps, ckpt_every, t0, grad_uT, grad_u0, grad_kappa,
                            grad_alpha, grad_params);
  p->noalloc = false;
  p->Pa = saved[0];
  p->zh = saved[1];
  p->aacc = saved[2];
  p->ahat = saved[3];
  p->gu = saved[4];
  p->seg = saved[5];
  p->G = (double*)saved[6];
  p->dcoef = saved[7];
  p->rp_acc = (double*)saved[8];
  p->thp = (double*)saved[9];
  p->red = (double*)saved[10];
  p->seg_steps = saved_seg;
  p->seg_cap = saved_cap;
  p->red_len = saved_red;
  return rc;
}

int64_t sfrde_workspace_bytes(sfrde_plan_t p) {
  if (!p) return fail(SFRDE_EINVAL, "plan is NULL");
  return (int64_t)p->bytes;
}

int sfrde_profile(sfrde_plan_t p, int32_t enable) {
  g_err.clear();
  if (!p) return fail(SFRDE_EINVAL, "plan is NULL");
  if (enable) {
    HIPCHECK(hipStreamSynchronize(p->stream));
    p->ev_used = 0;
    // Pre-create events for `enable` launches so that recording does not
    // create them inside a measured region.
    while (p->ev.size() < 2 * (size_t)enable) {
      hipEvent_t e;
      HIPCHECK(hipEventCreate(&e));
      p->ev.push_back(e);
    }
  }
  p->prof = enable != 0;
  return SFRDE_OK;
}

int sfrde_profile_read(sfrde_plan_t p, double* ms, int64_t* launches) {
  g_err.clear();
  if (!p || !ms || !launches) return fail(SFRDE_EINVAL, "NULL argument");
  HIPCHECK(hipStreamSynchronize(p->stream));
  for (int c = 0; c < KC_COUNT; ++c) {
    ms[c] = 0.0;
    launches[c] = 0;
  }
  for (size_t k = 0; k < p->ev_used; ++k) {
    float t = 0.f;
    HIPCHECK(hipEventElapsedTime(&t, p->ev[2 * k], p->ev[2 * k + 1]));
    ms[p->ev_class[k]] += double(t);
    launches[p->ev_class[k]] += 1;
  }
  return SFRDE_OK;
}

int sfrde_axis_eigenvalues(int32_t bc, int64_t n, double h, double* out) {
  g_err.clear();
  if (bc < 0 || bc > 2 || n < 2 || !(h > 0) || !out) return fail(SFRDE_EINVAL, "bad argument");
  for (int64_t k = 0; k < n; ++k) out[k] = axis_eigenvalue(bc, n, h, k);
  return SFRDE_OK;
}

int sfrde_eval_coefficients(int32_t scheme, double L, double dt, int32_t deriv, double* out6) {
  g_err.clear();
  if ((scheme != 0 && scheme != 1) || !(L >= 0) || !(dt > 0) || !out6)
    return fail(SFRDE_EINVAL, "bad argument");
  if (deriv)
    coef_derivs(scheme, L, dt, out6);
  else
    coef_values(scheme, L, dt, out6);
  return SFRDE_OK;
}

int sfrde_amplification(int32_t scheme, int64_t count, const double* x, const double* y,
                        double* r, void* hip_stream) {
  g_err.clear();
  if (scheme != SFRDE_SCHEME_P13 && scheme != SFRDE_SCHEME_EXP)
    return fail(SFRDE_EINVAL, "unknown scheme %d", scheme);
  if (count < 0 || count > (int64_t)1 << 36) return fail(SFRDE_EINVAL, "count out of range");
  if (count == 0) return SFRDE_OK;
  if (!x || !y || !r) return fail(SFRDE_EINVAL, "x, y and r must not be NULL");
  const unsigned blocks = (unsigned)((count + 255) / 256);
  hipLaunchKernelGGL(k_amplification, dim3(blocks), dim3(256), 0, (hipStream_t)hip_stream,
                     (int)scheme, (long long)count, x, y, r);
  HIPCHECK(hipGetLastError());
  return SFRDE_OK;
}

int sfrde_stability_boundary(int32_t scheme, int64_t ny, const double* y, int64_t ntheta,
                             double* roots, double* poly, void* hip_stream) {
  g_err.clear();
  if (scheme != SFRDE_SCHEME_P13 && scheme != SFRDE_SCHEME_EXP)
    return fail(SFRDE_EINVAL, "unknown scheme %d", scheme);
  if (ny < 0 || ntheta < 1 || ny > ((int64_t)1 << 30) || ntheta > ((int64_t)1 << 30) ||
      ny * ntheta > ((int64_t)1 << 34))
    return fail(SFRDE_EINVAL, "ny, ntheta out of range");
  if (ny == 0) return SFRDE_OK;
  if (!y || !roots) return fail(SFRDE_EINVAL, "y and roots must not be NULL");
  const long long total = (long long)ny * ntheta;
  const unsigned blocks = (unsigned)((total + 255) / 256);
  hipLaunchKernelGGL(k_stability_boundary, dim3(blocks), dim3(256), 0, (hipStream_t)hip_stream,
                     (int)scheme, (long long)ny, y, (long long)ntheta, roots, poly);
  HIPCHECK(hipGetLastError());
  return SFRDE_OK;
}

}  // extern "C"
