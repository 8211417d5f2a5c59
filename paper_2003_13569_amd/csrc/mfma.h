// Per-axis transforms on the matrix cores (gfx950 MFMA).
//
// Each axis matrix M (n x n, see kernels.h) has a reflection symmetry: with
// r(j) the mirrored index, M[k][r(j)] = +-M[k][j] (DCT-I, DST-I: sign (-1)^k),
// or M = C + S with C even and S odd under r (Hartley). Folding the input,
//   s_i = x[a_i] + x[b_i],  d_i = x[a_i] - x[b_i]   (pairs a_i, b_i = r(a_i)),
// splits the product into two half-size dense products E s and O d, and the
// outputs are recovered by an unfold: y_2m = (Es)_m, y_2m+1 = (Od)_m for
// DCT/DST, y_k = (Es)_k + (Od)_k and y_{N-k} = (Es)_k - (Od)_k for Hartley.
// That halves the multiply-adds of the dense product.
//
// The half-size matrices live in registers of a persistent block of 16
// waves: wave w owns 16 rows of E (w < RBe) or of O, for all K. Per tile of
// W lines the block folds the data in LDS, each wave runs its row block over
// all lines, results go back to LDS and are unfolded into the tile.
//
// FP32 fields: products on v_mfma_f32_16x16x32_bf16 with both operands split
// into three bf16 terms (x = x0 + x1 + x2, each the rounding of what is left)
// and the six products with term orders summing to at most 2, accumulated in
// FP32 from the smallest terms up: about the accuracy of an FP32 product.
// FP64 fields: v_mfma_f64_16x16x4_f64 on the unsplit values.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.h"

namespace sfrde {

constexpr int MF_THREADS = 1024;  // 16 waves
constexpr int MF_WAVES = 16;
constexpr int MF_KSMAX_F32 = 4;   // K <= 128 in steps of 32
constexpr int MF_KSMAX_F64 = 32;  // K <= 128 in steps of 4

struct MfmaAxisDev {
  const void* Afrag;      // fragment-ordered half matrices
  int n;                  // axis length
  int ns;                 // folded entries (pairs and fixed points)
  int periodic;           // Hartley fold (else DCT-I / DST-I)
  int hK;                 // folded length (multiple of 32)
  int RBe;                // 16-row blocks of E
  int RB;                 // 16-row blocks of E and O (<= 16)
  int fb_pitch;           // row pitch of the fold buffer (elements)
  int r_pitch;            // row pitch of the result buffer (elements)
  int fb_off;             // byte offset of the fold/result area in LDS
  int direct;             // unfold is the even/odd row interleave (DCT-I, DST-I)
};

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// Fold entry i: s_i = x[a] + x[b], d_i = x[a] - x[b]; b < 0 for a fixed point
// of the reflection (d_i = 0), a < 0 for padding (s_i = d_i = 0).
//   DCT-I / DST-I: pairs (i, n-1-i) for 2i+1 < n; the middle index when n is odd.
//   Hartley (N = n): 0 and N/2 are fixed; pairs (i, N-i) otherwise.
__device__ __forceinline__ void fold_pair(const MfmaAxisDev& ax, int i, int& a, int& b) {
  if (i >= ax.ns) {
    a = -1;
    b = -1;
    return;
  }
  a = i;
  if (!ax.periodic)
    b = 2 * i + 1 < ax.n ? ax.n - 1 - i : -1;
  else
    b = (i == 0 || 2 * i == ax.n) ? -1 : ax.n - i;
}

// Fold every line of one species' tile into fb: s rows then d rows, each
// [W][fb_pitch], eight consecutive i per work item.
template <typename T, int W>
__device__ __forceinline__ void mf_fold(const T* x, int pitch, const MfmaAxisDev& ax, T* fb) {
  const int items = W * (ax.hK / 8);
  for (int it = threadIdx.x; it < items; it += blockDim.x) {
    const int col = it % W;
    const int i0 = (it / W) * 8;
    T sv[8], dv[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      int a, b;
      fold_pair(ax, i0 + e, a, b);
      const T xa = a >= 0 ? x[a * pitch + col] : T(0);
      const T xb = b >= 0 ? x[b * pitch + col] : T(0);
      sv[e] = xa + xb;
      dv[e] = b >= 0 ? xa - xb : T(0);
    }
    T* ps = fb + col * ax.fb_pitch + i0;
    T* pd = fb + (W + col) * ax.fb_pitch + i0;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      ps[e] = sv[e];
      pd[e] = dv[e];
    }
  }
}

// Hartley unfold of the result rows R[row][col] into the tile x[k][col]:
// y_k = E_k + O_k for k <= N/2, y_k = E_{N-k} - O_{N-k} above.
template <typename T, int W>
__device__ __forceinline__ void mf_unfold(const T* R, const MfmaAxisDev& ax, int n, T* x, int pitch) {
  const int ne = n * W;
  const int obase = 16 * ax.RBe;
  for (int e = threadIdx.x; e < ne; e += blockDim.x) {
    const int k = e / W, col = e - k * W;
    const bool low = 2 * k <= n;
    const int kk = low ? k : n - k;
    const T ev = R[kk * ax.r_pitch + col], ov = R[(obase + kk) * ax.r_pitch + col];
    x[k * pitch + col] = low ? ev + ov : ev - ov;
  }
}

// ------------------------------------------------------------------ FP32
// Fold buffer: three bf16 terms of s and d, [term][half][col][fb_pitch]
// (bf16 bits), written once per element by the fold.
__device__ __forceinline__ void split_pair(float x, unsigned short& h0, unsigned short& h1,
                                           unsigned short& h2) {
  const __bf16 a = (__bf16)x;
  const float r1 = x - (float)a;
  const __bf16 b = (__bf16)r1;
  const float r2 = r1 - (float)b;
  const __bf16 c = (__bf16)r2;
  h0 = __builtin_bit_cast(unsigned short, a);
  h1 = __builtin_bit_cast(unsigned short, b);
  h2 = __builtin_bit_cast(unsigned short, c);
}

template <int W>
__device__ __forceinline__ void mf_fold_split(const float* x, int pitch, const MfmaAxisDev& ax,
                                              unsigned short* fb) {
  const int items = W * (ax.hK / 4);
  const int tstride = 2 * W * ax.fb_pitch;  // elements between terms
  for (int it = threadIdx.x; it < items; it += blockDim.x) {
    const int col = it % W;
    const int i0 = (it / W) * 4;
    unsigned short hs[3][4], hd[3][4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      int a, b;
      fold_pair(ax, i0 + e, a, b);
      const float xa = a >= 0 ? x[a * pitch + col] : 0.f;
      const float xb = b >= 0 ? x[b * pitch + col] : 0.f;
      split_pair(xa + xb, hs[0][e], hs[1][e], hs[2][e]);
      split_pair(b >= 0 ? xa - xb : 0.f, hd[0][e], hd[1][e], hd[2][e]);
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      const uint2 vs = make_uint2(hs[t][0] | ((unsigned)hs[t][1] << 16),
                                  hs[t][2] | ((unsigned)hs[t][3] << 16));
      const uint2 vd = make_uint2(hd[t][0] | ((unsigned)hd[t][1] << 16),
                                  hd[t][2] | ((unsigned)hd[t][3] << 16));
      *reinterpret_cast<uint2*>(fb + t * tstride + col * ax.fb_pitch + i0) = vs;
      *reinterpret_cast<uint2*>(fb + t * tstride + (W + col) * ax.fb_pitch + i0) = vd;
    }
  }
}

struct MfmaXfF32 {
  static constexpr int W = 32;
  const Geom* g;
  const MfmaAxisDev* ax;
  unsigned short* fb;
  bf16x8 A[MF_KSMAX_F32][3];
  int wave, lane;

  __device__ __forceinline__ MfmaXfF32(const Geom* g_, const MfmaAxisDev* ax_, float* fb_)
      : g(g_), ax(ax_), fb(reinterpret_cast<unsigned short*>(fb_)) {
    wave = threadIdx.x / 64;
    lane = threadIdx.x % 64;
    const uint4* src = reinterpret_cast<const uint4*>(ax->Afrag);
#pragma unroll
    for (int ks = 0; ks < MF_KSMAX_F32; ++ks)
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        uint4 v = make_uint4(0, 0, 0, 0);
        if (wave < ax->RB) v = src[((wave * MF_KSMAX_F32 + ks) * 3 + t) * 64 + lane];
        A[ks][t] = __builtin_bit_cast(bf16x8, v);
      }
  }

  __device__ __forceinline__ void operator()(float* buf, int S) {
    const int n = g->n, pitch = g->pitch;
    const int KS = ax->hK / 32;
    const int tstride = 2 * W * ax->fb_pitch;
    const bool isO = wave >= ax->RBe;
    for (int s = 0; s < S; ++s) {
      float* x = buf + s * n * pitch;
      mf_fold_split<W>(x, pitch, *ax, fb);
      __syncthreads();
      f32x4 acc[2];
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) acc[cb] = f32x4{0.f, 0.f, 0.f, 0.f};
      if (wave < ax->RB) {
        const int half = isO ? 1 : 0;
#pragma unroll
        for (int ks = 0; ks < MF_KSMAX_F32; ++ks) {
          if (ks < KS) {
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
              const unsigned short* bp = fb + (half * W + 16 * cb + lane % 16) * ax->fb_pitch +
                                         32 * ks + 8 * (lane / 16);
              const bf16x8 b0 = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(bp));
              const bf16x8 b1 =
                  __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(bp + tstride));
              const bf16x8 b2 =
                  __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(bp + 2 * tstride));
              f32x4 c = acc[cb];
              c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[ks][2], b0, c, 0, 0, 0);
              c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[ks][1], b1, c, 0, 0, 0);
              c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[ks][0], b2, c, 0, 0, 0);
              c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[ks][1], b0, c, 0, 0, 0);
              c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[ks][0], b1, c, 0, 0, 0);
              c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[ks][0], b0, c, 0, 0, 0);
              acc[cb] = c;
            }
          }
        }
      }
      if (ax->direct) {
        // DCT-I / DST-I: E row m is output 2m, O row m is output 2m + 1.
        if (wave < ax->RB) {
          const int mb = 16 * (isO ? wave - ax->RBe : wave) + 4 * (lane / 16);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int k = 2 * (mb + r) + (isO ? 1 : 0);
            if (k < n) {
#pragma unroll
              for (int cb = 0; cb < 2; ++cb) x[k * pitch + 16 * cb + lane % 16] = acc[cb][r];
            }
          }
        }
        __syncthreads();
      } else {
        float* R = reinterpret_cast<float*>(fb);
        __syncthreads();
        if (wave < ax->RB) {
#pragma unroll
          for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              R[(16 * wave + 4 * (lane / 16) + r) * ax->r_pitch + 16 * cb + lane % 16] = acc[cb][r];
        }
        __syncthreads();
        mf_unfold<float, W>(R, *ax, n, x, pitch);
        __syncthreads();
      }
    }
  }
};

// ------------------------------------------------------------------ FP64
struct MfmaXfF64 {
  static constexpr int W = 16;
  const Geom* g;
  const MfmaAxisDev* ax;
  double* fb;
  double A[MF_KSMAX_F64];
  int wave, lane;

  __device__ __forceinline__ MfmaXfF64(const Geom* g_, const MfmaAxisDev* ax_, double* fb_)
      : g(g_), ax(ax_), fb(fb_) {
    wave = threadIdx.x / 64;
    lane = threadIdx.x % 64;
    const double* src = reinterpret_cast<const double*>(ax->Afrag);
#pragma unroll
    for (int ks = 0; ks < MF_KSMAX_F64; ++ks)
      A[ks] = wave < ax->RB ? src[(wave * MF_KSMAX_F64 + ks) * 64 + lane] : 0.0;
  }

  __device__ __forceinline__ void operator()(double* buf, int S) {
    const int n = g->n, pitch = g->pitch;
    const int KS = ax->hK / 4;
    for (int s = 0; s < S; ++s) {
      double* x = buf + s * n * pitch;
      mf_fold<double, W>(x, pitch, *ax, fb);
      __syncthreads();
      f64x4 acc = f64x4{0.0, 0.0, 0.0, 0.0};
      if (wave < ax->RB) {
        const int half = wave < ax->RBe ? 0 : 1;
        const double* bp = fb + (half * W + lane % 16) * ax->fb_pitch + lane / 16;
#pragma unroll
        for (int ks = 0; ks < MF_KSMAX_F64; ++ks) {
          if (ks < KS) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A[ks], bp[4 * ks], acc, 0, 0, 0);
        }
      }
      // f64 16x16x4 result layout: lane l, register r holds row 4r + l/16, column l%16
      if (ax->direct) {
        // DCT-I / DST-I: E row m is output 2m, O row m is output 2m + 1.
        if (wave < ax->RB) {
          const bool isO = wave >= ax->RBe;
          const int mb = 16 * (isO ? wave - ax->RBe : wave) + lane / 16;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int k = 2 * (mb + 4 * r) + (isO ? 1 : 0);
            if (k < n) x[k * pitch + lane % 16] = acc[r];
          }
        }
        __syncthreads();
      } else {
        __syncthreads();
        if (wave < ax->RB) {
#pragma unroll
          for (int r = 0; r < 4; ++r)
            fb[(16 * wave + 4 * r + lane / 16) * ax->r_pitch + lane % 16] = acc[r];
        }
        __syncthreads();
        mf_unfold<double, W>(fb, *ax, n, x, pitch);
        __syncthreads();
      }
    }
  }
};

template <typename T>
struct MfmaXfSel;
template <>
struct MfmaXfSel<float> {
  using type = MfmaXfF32;
};
template <>
struct MfmaXfSel<double> {
  using type = MfmaXfF64;
};
template <typename T>
using MfmaXf = typename MfmaXfSel<T>::type;

// ------------------------------------------------------------------ kernels
// Persistent: block b handles tiles b, b + gridDim.x, ... The global loads of
// the next tile are issued before the current tile is computed.
// Prefetch depth (16-byte vectors per thread) where the registers allow it:
// the FP32 forward, single-axis and adjoint-X kernels; 0 loads in place.
template <typename T>
struct MfPrefetch {
  static constexpr int fwd = 0;
};
template <>
struct MfPrefetch<float> {
  static constexpr int fwd = 4;
};

template <typename T>
__global__ __launch_bounds__(MF_THREADS) void k_xstage_m(StageArgs<T> a, MfmaAxisDev ax) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* buf = reinterpret_cast<T*>(smem_raw);
  MfmaXf<T> xf(&a.g, &ax, reinterpret_cast<T*>(smem_raw + ax.fb_off));
  TilePrefetch<T, MfPrefetch<T>::fwd> pf;
  pf.issue(a.g, blockIdx.x, a.P, a.S);
  for (long long tile = blockIdx.x; tile < a.g.ntiles; tile += gridDim.x) {
    pf.commit(a.g, tile, a.P, buf, a.S);
    __syncthreads();
    pf.issue(a.g, tile + gridDim.x, a.P, a.S);
    run_x(a, buf, tile, xf);
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(MF_THREADS) void k_zstage_m(StageArgs<T> a, MfmaAxisDev ax) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* buf = reinterpret_cast<T*>(smem_raw);
  MfmaXf<T> xf(&a.g, &ax, reinterpret_cast<T*>(smem_raw + ax.fb_off));
  const T* src = a.src ? a.src : a.P;
  TilePrefetch<T, MfPrefetch<T>::fwd> pf;
  pf.issue(a.g, blockIdx.x, src, a.S);
  for (long long tile = blockIdx.x; tile < a.g.ntiles; tile += gridDim.x) {
    pf.commit(a.g, tile, src, buf, a.S);
    __syncthreads();
    pf.issue(a.g, tile + gridDim.x, src, a.S);
    run_z(a, buf, tile, xf);
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(MF_THREADS) void k_xadj_m(StageArgs<T> a, MfmaAxisDev ax) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* buf = reinterpret_cast<T*>(smem_raw);
  MfmaXf<T> xf(&a.g, &ax, reinterpret_cast<T*>(smem_raw + ax.fb_off));
  double pacc[MAX_PARAMS];
  for (int k = 0; k < MAX_PARAMS; ++k) pacc[k] = 0.0;
  TilePrefetch<T, MfPrefetch<T>::fwd> pf;
  pf.issue(a.g, blockIdx.x, a.P, a.S);
  for (long long tile = blockIdx.x; tile < a.g.ntiles; tile += gridDim.x) {
    pf.commit(a.g, tile, a.P, buf, a.S);
    __syncthreads();
    pf.issue(a.g, tile + gridDim.x, a.P, a.S);
    run_xadj(a, buf, tile, xf, pacc);
    __syncthreads();
  }
  if (a.rp_acc) block_add_partials(reinterpret_cast<double*>(smem_raw), pacc, a.rxn.np, a.rp_acc);
}

template <typename T>
__global__ __launch_bounds__(MF_THREADS) void k_zadj_m(StageArgs<T> a, MfmaAxisDev ax) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* buf = reinterpret_cast<T*>(smem_raw);
  MfmaXf<T> xf(&a.g, &ax, reinterpret_cast<T*>(smem_raw + ax.fb_off));
  TilePrefetch<T, 0> pf;
  pf.issue(a.g, blockIdx.x, a.P, a.S);
  for (long long tile = blockIdx.x; tile < a.g.ntiles; tile += gridDim.x) {
    pf.commit(a.g, tile, a.P, buf, a.S);
    __syncthreads();
    pf.issue(a.g, tile + gridDim.x, a.P, a.S);
    run_zadj(a, buf, tile, xf);
    __syncthreads();
  }
}

// One transform along one axis, src -> dst (may alias), optional Neumann
// point weights before (divide) or after (multiply).
template <typename T>
__global__ __launch_bounds__(MF_THREADS) void k_single_m(SingleArgs<T> a, MfmaAxisDev ax) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* buf = reinterpret_cast<T*>(smem_raw);
  MfmaXf<T> xf(&a.g, &ax, reinterpret_cast<T*>(smem_raw + ax.fb_off));
  const Geom& g = a.g;
  const int ne = g.n * g.W;
  TilePrefetch<T, MfPrefetch<T>::fwd> pf;
  pf.issue(g, blockIdx.x, a.src, a.S);
  for (long long tile = blockIdx.x; tile < g.ntiles; tile += gridDim.x) {
    pf.commit(g, tile, a.src, buf, a.S);
    __syncthreads();
    pf.issue(g, tile + gridDim.x, a.src, a.S);
    const TileRef tr = tile_ref(g, tile);
    if (a.pre_divide_w) {
      for (int e = threadIdx.x; e < ne; e += blockDim.x) {
        int j, w;
        unpack(g, e, j, w);
        long long idx;
        if (!elem(g, tr, j, w, idx)) continue;
        const T wt = T(point_weight(idx, a.n0, a.n1, a.n2));
        for (int s = 0; s < a.S; ++s) buf[(s * g.n + j) * g.pitch + w] /= wt;
      }
      __syncthreads();
    }
    xf(buf, a.S);
    if (a.post_multiply_w) {
      for (int e = threadIdx.x; e < ne; e += blockDim.x) {
        int j, w;
        unpack(g, e, j, w);
        long long idx;
        if (!elem(g, tr, j, w, idx)) continue;
        const T wt = T(point_weight(idx, a.n0, a.n1, a.n2));
        for (int s = 0; s < a.S; ++s) buf[(s * g.n + j) * g.pitch + w] *= wt;
      }
      __syncthreads();
    }
    store_tile_fast(g, tile, buf, a.dst, a.S);
    __syncthreads();
  }
}

}  // namespace sfrde
