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
// The half-size matrices live in registers of a persistent block of 8
// waves, one block per CU: wave w owns the 16-row blocks 2w and 2w + 1 of E
// (block index < RBe) or of O, for all K. Per tile of W lines the block folds
// the data in LDS, each wave runs its row blocks over all lines, results go
// back to LDS and are unfolded into the tile.
//
// FP32 fields: products on v_mfma_f32_16x16x32_f16 with both operands split
// into two binary16 terms after a per-column power-of-two scaling, three
// products accumulated in FP32: about the accuracy of an FP32 product.
// FP64 fields: v_mfma_f64_16x16x4_f64 on the unsplit values.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "kernels.h"

namespace sfrde {

constexpr int MF_WAVES = 16;      // 16-row blocks of E and O at most (two per wave)
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
  int nfb;                // FP32 fold buffers in LDS (2 where they fit on the x axis, else 1)
};

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
// Products on v_mfma_f32_16x16x32_f16. Both operands are split into two
// binary16 terms, v = v0 + v1 with v0 the rounding of v and v1 the rounding
// of what is left, and the three products A0 X0 + A0 X1 + A1 X0 are
// accumulated in FP32 (the dropped A1 X1 is below 2^-22 of the column
// scale). The matrices hold bounded entries (|a| <= sqrt 2); each folded data
// column is scaled by a power of two that puts its largest magnitude in
// [2^14, 2^15), so neither term leaves the binary16 range, and the results
// are scaled back exactly.
//
// Fold buffer (LDS, binary16 bits): [term][half s|d][col][F32_FBP], then the
// W inverse column scales as floats. F32_FBP = 136 leaves room for folded
// lengths up to 128 and keeps the 16-byte accesses free of bank conflicts.
constexpr int F32_FBP = 136;
constexpr int f32_fold_bytes(int W) { return 2 * 2 * W * F32_FBP * 2 + W * 4; }

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef _Float16 h2v __attribute__((ext_vector_type(2)));

// Two scaled floats -> packed binary16 head and tail terms.
__device__ __forceinline__ void split2_f16(float x0, float x1, float sc, unsigned& t0,
                                           unsigned& t1) {
  const f2v x = {x0 * sc, x1 * sc};
  const h2v a = __builtin_convertvector(x, h2v);
  const f2v r = x - __builtin_convertvector(a, f2v);
  const h2v b = __builtin_convertvector(r, h2v);
  t0 = __builtin_bit_cast(unsigned, a);
  t1 = __builtin_bit_cast(unsigned, b);
}

// Maximum over the 16 lanes of a DPP row (lanes 16r .. 16r+15).
__device__ __forceinline__ float row16_max(float m) {
  m = fmaxf(m, __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
                                             0, __builtin_bit_cast(int, m), 0x128, 0xf, 0xf, false)));
  m = fmaxf(m, __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
                                             0, __builtin_bit_cast(int, m), 0x124, 0xf, 0xf, false)));
  m = fmaxf(m, __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
                                             0, __builtin_bit_cast(int, m), 0x122, 0xf, 0xf, false)));
  m = fmaxf(m, __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
                                             0, __builtin_bit_cast(int, m), 0x121, 0xf, 0xf, false)));
  return m;
}

// Eight waves; wave w owns row blocks 2w and 2w + 1 (of E, then of O), so
// one 512-thread block per CU has 256 registers per lane for the fragments
// and the prefetched tile. W = 32 lines (128-byte rows on strided axes).
template <int W_, bool XAX_>
struct MfmaXfF32 {
  static constexpr int W = W_;
  static constexpr bool XAX = XAX_;  // x-axis tiles (every species) rather than strided ones
  static constexpr int THREADS = 512;
  static constexpr int MIN_WAVES_PER_EU = 2;  // one block per CU, 256 registers per lane
  static constexpr int P = W + 1;             // LDS row pitch of the tile
  static constexpr int FBP = F32_FBP;
  static constexpr int TS = 2 * W * F32_FBP;  // binary16 elements between the two terms
  static constexpr int FOLD_THREADS = 16 * W; // one 16-lane row per column
  static constexpr int CB = W / 16;           // 16-column blocks
  // Fold buffers: x tiles (every species) alternate two where LDS allows
  // (ax->nfb), so that one species' fold can run while other waves still
  // multiply the previous one.
  static constexpr int FBH = f32_fold_bytes(W) / 2;  // binary16 elements per buffer
  const MfmaAxisDev* ax;
  unsigned short* fb0;
  unsigned short* fb;  // the buffer in use
  float* scl;          // its inverse column scales
  f16x8 A[2][MF_KSMAX_F32][2];
  int n, KS;
  int nrb;      // row blocks of this wave (0..2)
  bool shareB;  // both row blocks read the same fold half
  bool direct;
  int bofs[2];  // B-fragment offsets in fb per row block
  // fold work item of this thread: column col, entries i0 .. i0+7
  bool ffast;
  int i0, col, fa, fbb;
  // first output row of this lane's results (direct unfold), per row block
  int rmask[2], orow[2];

  __device__ __forceinline__ MfmaXfF32(const Geom*, const MfmaAxisDev* ax_, float* fb_)
      : ax(ax_), fb0(reinterpret_cast<unsigned short*>(fb_)) {
    use(0);
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    n = ax->n;
    KS = ax->hK >> 5;
    direct = ax->direct != 0;
    const int rb0 = 2 * wave;
    nrb = ax->RB - rb0;
    nrb = nrb < 0 ? 0 : (nrb > 2 ? 2 : nrb);
    const uint4* src = reinterpret_cast<const uint4*>(ax->Afrag);
    bool isO[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int rb = rb0 + h;
#pragma unroll
      for (int ks = 0; ks < MF_KSMAX_F32; ++ks)
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          uint4 v = make_uint4(0, 0, 0, 0);
          if (h < nrb) v = src[((rb * MF_KSMAX_F32 + ks) * 2 + t) * 64 + lane];
          A[h][ks][t] = __builtin_bit_cast(f16x8, v);
        }
      isO[h] = rb >= ax->RBe;
      bofs[h] = ((isO[h] ? W : 0) + lane % 16) * FBP + 8 * (lane / 16);
      // direct unfold: E row m -> output 2m, O row m -> output 2m + 1
      const int mb = 16 * (isO[h] ? rb - ax->RBe : rb) + 4 * (lane / 16);
      const int row0 = 2 * mb + (isO[h] ? 1 : 0);
      orow[h] = row0;
      rmask[h] = 0;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (h < nrb && row0 + 2 * r < n) rmask[h] |= 1 << r;
    }
    shareB = nrb < 2 || isO[0] == isO[1];
    // Wait for the fragment loads here: left pending, they would make the
    // compiler wait for every outstanding load before the first product of
    // each tile, prefetches included. (gfx9 s_waitcnt: vmcnt 0, others max.)
    __builtin_amdgcn_s_waitcnt(0x0F70);
    // fold item; entries past the folded length come out as zeros
    col = (threadIdx.x >> 4) & (W - 1);
    i0 = (threadIdx.x & 15) << 3;
    const int bstart = ax->periodic ? n : n - 1;  // partner of entry i is bstart - i
    ffast = ax->periodic ? (i0 >= 1 && 2 * (i0 + 7) < n) : (2 * (i0 + 7) + 1 < n);
    fa = i0 * P + col;
    fbb = (bstart - i0) * P + col;
  }

  // Select fold buffer b mod nfb for the next fold and products.
  __device__ __forceinline__ void use(int b) {
    fb = fb0 + (XAX && ax->nfb > 1 ? (b & 1) * FBH : 0);
    scl = reinterpret_cast<float*>(fb + 2 * TS);
  }
  __device__ __forceinline__ bool two_buffers() const { return XAX && ax->nfb > 1; }

  // Entries 64 and up of the fold buffer are stored rotated by four within
  // each group of eight (item e of a work item at i0 >= 64 holds entry
  // i0 + (e ^ 4)); the host orders the matrix fragments the same way, so the
  // products are unchanged. The fold's LDS reads then never hit one bank
  // twice: rows 64 apart share a bank at any tile pitch, and the two halves
  // of a 16-lane row would otherwise read such rows at once.
  __device__ __forceinline__ void fold(const float* x) {
    if ((int)threadIdx.x >= FOLD_THREADS) return;
    float sv[8], dv[8];
    const int rot = (threadIdx.x & 8) ? 4 : 0;  // i0 >= 64
    if (ffast) {
      const float* xa0 = x + fa + rot * P;   // items 0..3: entries i0 + rot + e
      const float* xa1 = x + fa - rot * P;   // items 4..7: entries i0 - rot + e
      const float* xb0 = x + fbb - rot * P;  // their partners
      const float* xb1 = x + fbb + rot * P;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float xa = e < 4 ? xa0[e * P] : xa1[e * P];
        const float xb = e < 4 ? xb0[-e * P] : xb1[-e * P];
        sv[e] = xa + xb;
        dv[e] = xa - xb;
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        int a, b;
        fold_pair(*ax, i0 + (e ^ rot), a, b);
        const float xa = a >= 0 ? x[a * P + col] : 0.f;
        const float xb = b >= 0 ? x[b * P + col] : 0.f;
        sv[e] = xa + xb;
        dv[e] = b >= 0 ? xa - xb : 0.f;
      }
    }
    fold_store(sv, dv);
  }

  // Fold from registers: v[0], v[1] hold entries i0 .. i0+7 of this thread's
  // line, v[2], v[3] entries n-8-i0 .. n-1-i0 (DCT-I / DST-I pairs i, n-1-i;
  // items past the folded length are padding), each pair of float4 swapped
  // where i0 >= 64 (the rotated order of fold()).
  __device__ __forceinline__ void fold_regs(const float4 (&v)[4]) {
    float sv[8], dv[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float xa = vget<float>(v[e >> 2], e & 3);
      const float xb = vget<float>(v[2 + ((7 - e) >> 2)], (7 - e) & 3);
      sv[e] = ffast ? xa + xb : 0.f;
      dv[e] = ffast ? xa - xb : 0.f;
    }
    fold_store(sv, dv);
  }

  // Column scale, binary16 split and store of one fold item.
  __device__ __forceinline__ void fold_store(const float (&sv)[8], const float (&dv)[8]) {
    float m = 0.f;
#pragma unroll
    for (int e = 0; e < 8; ++e) m = fmaxf(m, fmaxf(fabsf(sv[e]), fabsf(dv[e])));
    m = row16_max(m);
    int k = 15 - __builtin_amdgcn_frexp_expf(m);
    k = k < -126 ? -126 : (k > 126 ? 126 : k);
    const float sc = __builtin_amdgcn_ldexpf(1.f, k);
    if ((threadIdx.x & 15) == 0) scl[col] = __builtin_amdgcn_ldexpf(1.f, -k);
    unsigned s0[4], s1[4], d0[4], d1[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      split2_f16(sv[2 * q], sv[2 * q + 1], sc, s0[q], s1[q]);
      split2_f16(dv[2 * q], dv[2 * q + 1], sc, d0[q], d1[q]);
    }
    unsigned short* ps = fb + col * FBP + i0;
    unsigned short* pd = ps + W * FBP;
    *reinterpret_cast<uint4*>(ps) = make_uint4(s0[0], s0[1], s0[2], s0[3]);
    *reinterpret_cast<uint4*>(ps + TS) = make_uint4(s1[0], s1[1], s1[2], s1[3]);
    *reinterpret_cast<uint4*>(pd) = make_uint4(d0[0], d0[1], d0[2], d0[3]);
    *reinterpret_cast<uint4*>(pd + TS) = make_uint4(d1[0], d1[1], d1[2], d1[3]);
  }

  __device__ __forceinline__ static f16x8 frag(const unsigned short* p) {
    return __builtin_bit_cast(f16x8, *reinterpret_cast<const uint4*>(p));
  }

  __device__ __forceinline__ void products(f32x4 (&acc)[2][CB]) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) acc[h][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
    if (nrb == 0) return;
    if (!XAX && nrb == 2 && shareB) {
      // both row blocks read the same fragments: the 2 CB accumulators are
      // independent, so consecutive products never wait on one another
      // (same summation order per accumulator as below)
#pragma unroll
      for (int ks = 0; ks < MF_KSMAX_F32; ++ks) {
        if (ks >= KS) break;
        f16x8 b0[CB], b1[CB];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
          const int off = 16 * cb * FBP + 32 * ks;
          b0[cb] = frag(fb + bofs[0] + off);
          b1[cb] = frag(fb + bofs[0] + off + TS);
        }
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
          for (int h = 0; h < 2; ++h)
            acc[h][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A[h][ks][1], b0[cb], acc[h][cb], 0, 0, 0);
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
          for (int h = 0; h < 2; ++h)
            acc[h][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A[h][ks][0], b1[cb], acc[h][cb], 0, 0, 0);
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
          for (int h = 0; h < 2; ++h)
            acc[h][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A[h][ks][0], b0[cb], acc[h][cb], 0, 0, 0);
      }
    } else {
#pragma unroll
    for (int ks = 0; ks < MF_KSMAX_F32; ++ks) {
      if (ks >= KS) break;
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        const int off = 16 * cb * FBP + 32 * ks;
        f16x8 b0 = frag(fb + bofs[0] + off), b1 = frag(fb + bofs[0] + off + TS);
        acc[0][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A[0][ks][1], b0, acc[0][cb], 0, 0, 0);
        acc[0][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A[0][ks][0], b1, acc[0][cb], 0, 0, 0);
        acc[0][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A[0][ks][0], b0, acc[0][cb], 0, 0, 0);
        if (nrb == 2) {
          if (!shareB) {
            b0 = frag(fb + bofs[1] + off);
            b1 = frag(fb + bofs[1] + off + TS);
          }
          acc[1][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A[1][ks][1], b0, acc[1][cb], 0, 0, 0);
          acc[1][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A[1][ks][0], b1, acc[1][cb], 0, 0, 0);
          acc[1][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A[1][ks][0], b0, acc[1][cb], 0, 0, 0);
        }
      }
    }
    }
    const int lane = threadIdx.x % 64;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      const float inv = scl[16 * cb + lane % 16];
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[h][cb][r] *= inv;
    }
  }

  // DCT-I / DST-I transform of one species' strided tile x with the results
  // written straight to global memory: row k of the tile to g + k inner (16
  // lanes write 64 contiguous bytes; x tiles, whose lines are n apart, never
  // take this path). The tile in LDS is left as it was.
  __device__ __forceinline__ void to_global(const float* x, float* g, long long inner) {
    fold(x);
    __syncthreads();
    f32x4 acc[2][CB];
    products(acc);
    const int lane = threadIdx.x % 64;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      float* gr = g + orow[h] * inner + lane % 16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (rmask[h] & (1 << r)) {
#pragma unroll
          for (int cb = 0; cb < CB; ++cb) gr[2 * r * inner + 16 * cb] = acc[h][cb][r];
        }
      }
    }
  }

  __device__ __forceinline__ void operator()(float* buf, int S) {
    for (int s = 0; s < S; ++s) {
      float* x = buf + s * n * P;
      use(s);
      fold(x);
      __syncthreads();
      // With two buffers the next species' fold (other rows of the tile, the
      // other buffer) needs no barrier after these products; the barrier
      // after the last species covers every result.
      mfma_write(x, !two_buffers() || s == S - 1);
    }
    use(0);
  }

  // Products of the folded data in fb and their unfold into the tile x;
  // sync: a barrier after the results (the unfold path always has one).
  __device__ __forceinline__ void mfma_write(float* x, bool sync = true) {
    const int lane = threadIdx.x % 64;
    {
      f32x4 acc[2][CB];
      products(acc);
      if (direct) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          float* xr = x + orow[h] * P + lane % 16;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            if (rmask[h] & (1 << r)) {
#pragma unroll
              for (int cb = 0; cb < CB; ++cb) xr[2 * r * P + 16 * cb] = acc[h][cb][r];
            }
          }
        }
        if (sync) __syncthreads();
      } else {
        float* R = reinterpret_cast<float*>(fb);
        const int rb0 = 2 * (threadIdx.x / 64);
        __syncthreads();
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          if (h < nrb) {
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
#pragma unroll
              for (int r = 0; r < 4; ++r)
                R[(16 * (rb0 + h) + 4 * (lane / 16) + r) * ax->r_pitch + 16 * cb + lane % 16] =
                    acc[h][cb][r];
          }
        }
        __syncthreads();
        mf_unfold<float, W>(R, *ax, n, x, P);
        __syncthreads();
      }
    }
  }
};

// ------------------------------------------------------------------ FP64
// Eight waves; wave w owns row blocks 2w and 2w + 1 (of E, then of O) for all
// K, 2 x 32 fragments = 128 registers per lane, with one 512-thread block per
// CU (256 registers per lane). Each row block runs two accumulation chains
// (even and odd ks), so a wave keeps four MFMA chains in flight.
struct MfmaXfF64 {
  static constexpr int W = 16;
  static constexpr int THREADS = 512;
  static constexpr int MIN_WAVES_PER_EU = 2;  // one block per CU, 256 registers per lane
  static constexpr bool XAX = false;          // one engine for every axis (tiles: TileIOF64 or generic)
  static constexpr int FOLD_E = 4;            // fold entries per work item
  const Geom* g;
  const MfmaAxisDev* ax;
  double* fb;
  double A[2][MF_KSMAX_F64];
  int wave, lane, nrb;
  bool isO[2];
  int bofs[2];  // B-fragment offsets in fb per row block

  __device__ __forceinline__ MfmaXfF64(const Geom* g_, const MfmaAxisDev* ax_, double* fb_)
      : g(g_), ax(ax_), fb(fb_) {
    wave = threadIdx.x / 64;
    lane = threadIdx.x % 64;
    const int rb0 = 2 * wave;
    nrb = ax->RB - rb0;
    nrb = nrb < 0 ? 0 : (nrb > 2 ? 2 : nrb);
    const double* src = reinterpret_cast<const double*>(ax->Afrag);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
      for (int ks = 0; ks < MF_KSMAX_F64; ++ks)
        A[h][ks] = h < nrb ? src[((rb0 + h) * MF_KSMAX_F64 + ks) * 64 + lane] : 0.0;
      isO[h] = rb0 + h >= ax->RBe;
      bofs[h] = ((isO[h] ? W : 0) + lane % 16) * ax->fb_pitch + lane / 16;
    }
  }

  // Fold of one species' tile into fb (s rows then d rows, [W][fb_pitch]),
  // FOLD_E consecutive entries per work item, every thread taking part.
  __device__ __forceinline__ void fold(const double* x, int pitch) {
    const int items = W * (ax->hK / FOLD_E);
    for (int it = threadIdx.x; it < items; it += THREADS) {
      const int col = it % W;
      const int i0 = (it / W) * FOLD_E;
      double sv[FOLD_E], dv[FOLD_E];
#pragma unroll
      for (int e = 0; e < FOLD_E; ++e) {
        int a, b;
        fold_pair(*ax, i0 + e, a, b);
        const double xa = a >= 0 ? x[a * pitch + col] : 0.0;
        const double xb = b >= 0 ? x[b * pitch + col] : 0.0;
        sv[e] = xa + xb;
        dv[e] = b >= 0 ? xa - xb : 0.0;
      }
      double* ps = fb + col * ax->fb_pitch + i0;
      double* pd = fb + (W + col) * ax->fb_pitch + i0;
#pragma unroll
      for (int e = 0; e < FOLD_E; e += 2) {
        *reinterpret_cast<double2*>(ps + e) = make_double2(sv[e], sv[e + 1]);
        *reinterpret_cast<double2*>(pd + e) = make_double2(dv[e], dv[e + 1]);
      }
    }
  }

  __device__ __forceinline__ void operator()(double* buf, int S) {
    const int n = g->n, pitch = g->pitch;
    const int KS = ax->hK / 4;
    for (int s = 0; s < S; ++s) {
      double* x = buf + s * n * pitch;
      fold(x, pitch);
      __syncthreads();
      f64x4 acc[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) acc[h] = f64x4{0.0, 0.0, 0.0, 0.0};
      if (nrb > 0) {
        // two chains per row block over even and odd ks (KS is a multiple of
        // 8: the folded length is a multiple of 32)
        f64x4 acc1[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) acc1[h] = f64x4{0.0, 0.0, 0.0, 0.0};
        const double* bp0 = fb + bofs[0];
        const double* bp1 = fb + bofs[1];
#pragma unroll
        for (int ks = 0; ks < MF_KSMAX_F64; ks += 2) {
          if (ks < KS) {
            const double b00 = bp0[4 * ks], b01 = bp0[4 * ks + 4];
            const double b10 = bp1[4 * ks], b11 = bp1[4 * ks + 4];
            acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(A[0][ks], b00, acc[0], 0, 0, 0);
            acc1[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(A[0][ks + 1], b01, acc1[0], 0, 0, 0);
            if (nrb == 2) {
              acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(A[1][ks], b10, acc[1], 0, 0, 0);
              acc1[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(A[1][ks + 1], b11, acc1[1], 0, 0, 0);
            }
          }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) acc[h] = acc[h] + acc1[h];
      }
      // f64 16x16x4 result layout: lane l, register r holds row 4r + l/16, column l%16
      if (ax->direct) {
        // DCT-I / DST-I: E row m is output 2m, O row m is output 2m + 1.
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          if (h < nrb) {
            const int rbl = 2 * wave + h - (isO[h] ? ax->RBe : 0);
            const int mb = 16 * rbl + lane / 16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int k = 2 * (mb + 4 * r) + (isO[h] ? 1 : 0);
              if (k < n) x[k * pitch + lane % 16] = acc[h][r];
            }
          }
        }
        __syncthreads();
      } else {
        __syncthreads();
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          if (h < nrb) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
              fb[(16 * (2 * wave + h) + 4 * r + lane / 16) * ax->r_pitch + lane % 16] = acc[h][r];
          }
        }
        __syncthreads();
        mf_unfold<double, W>(fb, *ax, n, x, pitch);
        __syncthreads();
      }
    }
  }
};

// Engines per field type: the x axis (tiles of every species) and the
// strided axes.
template <typename T>
struct XfSel;
template <>
struct XfSel<float> {
  using X = MfmaXfF32<32, true>;
  using Z = MfmaXfF32<32, false>;
};
template <>
struct XfSel<double> {
  using X = MfmaXfF64;
  using Z = MfmaXfF64;
};
template <typename T>
using XfX = typename XfSel<T>::X;
template <typename T>
using XfZ = typename XfSel<T>::Z;

// ------------------------------------------------------------------ tile movement
// FP32 engine tiles move in 16-byte vectors with per-thread offsets from the
// tile base (full tiles, 16-byte aligned fields, the shapes below); other
// tiles use the generic paths of kernels.h.
//
// Strided axis (W = 32, one species per tile, n a multiple of 64 up to 256):
// thread t moves rows row0(t) + 64k, lanes 4(t%8) .. +3.
// x axis (W = 16 lines, every species, n in {64, 128, 256}, 128 <= S n <= 512): a wave moves
// 16 consecutive vectors of each of 4 lines, so that the four scalar LDS
// writes of a vector land in distinct banks across the wave.
template <typename T, int W>
struct TileIO {
  __device__ __forceinline__ static void issue(const Geom&, const TileRef&, const T*, float4*) {}
  __device__ __forceinline__ static void commit(const Geom&, const float4*, T*) {}
  __device__ __forceinline__ static void store(const Geom&, const TileRef&, const T*, T*) {}
};

template <>
struct TileIO<float, 32> {
  static constexpr int P = 33, VPR = 8, RSTEP = 512 / VPR, MAXK = 4;
  // Wave w moves rows 4w .. 4w+3 and 4w+32 .. 4w+35 (8 lanes per row): with
  // the pitch of 33 floats the four scalar LDS accesses of a vector then hit
  // 64 distinct banks across the wave (rows r and r+4 would collide).
  __device__ __forceinline__ static int row0() {
    const int l = threadIdx.x & 63, rr = l >> 3;
    return 4 * (int)(threadIdx.x >> 6) + (rr & 3) + 32 * (rr >> 2);
  }
  __device__ __forceinline__ static int lane4() { return (threadIdx.x % VPR) * 4; }
  __device__ __forceinline__ static void issue(const Geom& g, const TileRef& tr, const float* src,
                                               float4* v) {
    const int r0 = row0(), w4 = lane4();
    const long long inner = g.inner;
    const float* sp = src + tr.base + r0 * inner + w4;
    // straight-line loads (rows past n repeat row block 0), so that the
    // compiler's wait counts stay exact
#pragma unroll
    for (int k = 0; k < MAXK; ++k)
      v[k] = *reinterpret_cast<const float4*>(sp + (64 * k < g.n ? k : 0) * RSTEP * inner);
  }
  __device__ __forceinline__ static void commit(const Geom& g, const float4* v, float* buf) {
    const int r0 = row0(), w4 = lane4();
#pragma unroll
    for (int k = 0; k < MAXK; ++k)
      if (64 * k < g.n) {
        float* b = buf + (r0 + RSTEP * k) * P + w4;
        b[0] = v[k].x;
        b[1] = v[k].y;
        b[2] = v[k].z;
        b[3] = v[k].w;
      }
  }
  __device__ __forceinline__ static void store(const Geom& g, const TileRef& tr, const float* buf,
                                               float* dst) {
    const int r0 = row0(), w4 = lane4();
    const long long inner = g.inner;
    float* dp = dst + tr.base + r0 * inner + w4;
    // straight-line stores: rows past n store row block 0 again (same values)
#pragma unroll
    for (int k = 0; k < MAXK; ++k) {
      const int kk = 64 * k < g.n ? k : 0;
      const float* b = buf + (r0 + RSTEP * kk) * P + w4;
      *reinterpret_cast<float4*>(dp + kk * RSTEP * inner) = make_float4(b[0], b[1], b[2], b[3]);
    }
  }
};

// x-axis tiles (inner == 1): W lines of every species. Vector v of species
// s: 16 consecutive vectors of each of 4 lines per 64 vectors, so that the
// four scalar LDS writes of a vector land in distinct banks across a wave.
template <int W>
struct XTileIO {
  static constexpr int P = W + 1;
  static constexpr int MAXV = W / 4;  // vectors per thread: S * W * n / 4 / 512 <= W / 4
  __device__ __forceinline__ static int log2n64(const Geom& g) {
    return g.n == 256 ? 2 : (g.n == 128 ? 1 : 0);
  }
  __device__ __forceinline__ static void coords(const Geom& g, int s, int v, int& go, int& lo) {
    const int lg = log2n64(g);
    const int c16 = v & 15, l4 = (v >> 4) & 3, rest = v >> 6;
    const int line = 4 * (rest >> lg) + l4;
    const int j = 4 * (16 * (rest & ((1 << lg) - 1)) + c16);
    go = line * g.n + j;
    lo = (s * g.n + j) * P + line;
  }
  // log2 of the vectors per species, W n / 4
  __device__ __forceinline__ static int vshift(const Geom& g) {
    return log2n64(g) + (W == 32 ? 9 : 8);
  }
  __device__ __forceinline__ static void issue(const Geom& g, const TileRef& tr, const float* src,
                                               float4* v) {
    const int sh = vshift(g);
    const int nv = g.spt << sh;  // vectors in the tile, a multiple of 512
#pragma unroll
    for (int k = 0; k < MAXV; ++k) {
      // straight-line loads (vectors past the tile repeat the first block)
      const int q = threadIdx.x + (512 * k < nv ? 512 * k : 0), s = q >> sh;
      int go, lo;
      coords(g, s, q & ((1 << sh) - 1), go, lo);
      v[k] = *reinterpret_cast<const float4*>(src + s * g.total + tr.base + go);
    }
  }
  __device__ __forceinline__ static void commit(const Geom& g, const float4* v, float* buf) {
    const int sh = vshift(g);
#pragma unroll
    for (int k = 0; k < MAXV; ++k) {
      const int q = threadIdx.x + 512 * k, s = q >> sh;
      if (s < g.spt) {
        int go, lo;
        coords(g, s, q & ((1 << sh) - 1), go, lo);
        float* b = buf + lo;
        b[0] = v[k].x;
        b[P] = v[k].y;
        b[2 * P] = v[k].z;
        b[3 * P] = v[k].w;
      }
    }
  }
  __device__ __forceinline__ static void store(const Geom& g, const TileRef& tr, const float* buf,
                                               float* dst) {
    const int sh = vshift(g);
    const int nv = g.spt << sh;
#pragma unroll
    for (int k = 0; k < MAXV; ++k) {
      // straight-line stores (vectors past the tile store the first block again)
      const int q = threadIdx.x + (512 * k < nv ? 512 * k : 0), s = q >> sh;
      int go, lo;
      coords(g, s, q & ((1 << sh) - 1), go, lo);
      const float* b = buf + lo;
      *reinterpret_cast<float4*>(dst + s * g.total + tr.base + go) =
          make_float4(b[0], b[P], b[2 * P], b[3 * P]);
    }
  }
};

// Adjoint reaction on an x tile in the XTileIO layout (every thread takes 4
// consecutive points of a line, all species): the stored stage values are
// read as vectors and the Neumann point weights formed from the coordinates.
template <int NS, bool WP = true>
__device__ __forceinline__ void xadj_reaction_vec(const StageArgs<float>& a, float* buf,
                                                  long long tile, double* pacc) {
  using IO = XTileIO<32>;
  const Geom& g = a.g;
  const TileRef tr = tile_ref(g, tile);
  const bool want_p = WP && a.rp_acc != nullptr;  // WP = false: never (host-checked)
  const int sh = IO::vshift(g);  // vectors per species 2^sh, a multiple of 512
  const int n = g.n;
  const int line0 = (int)(tile * 32);  // line index = y + n1 z (< 2^20)
  const int n1 = (int)a.n1, n2 = (int)a.n2;
  const bool three = n2 > 1;
  const int nv = 1 << sh;
  const float* sp = a.st_phys + (long long)a.mode * NS * g.total + tr.base;
  // the stored stage values of the next vector are loaded while this one is
  // computed (past the last vector the last one is loaded again)
  float4 cur[NS], nxt[NS];
  {
    int go, lo;
    IO::coords(g, 0, threadIdx.x, go, lo);
#pragma unroll
    for (int s = 0; s < NS; ++s)
      cur[s] = *reinterpret_cast<const float4*>(sp + (long long)s * g.total + go);
  }
#pragma unroll 1
  for (int q = threadIdx.x; q < nv; q += 512) {
    {
      const int qn = q + 512 < nv ? q + 512 : q;
      int go, lo;
      IO::coords(g, 0, qn, go, lo);
#pragma unroll
      for (int s = 0; s < NS; ++s)
        nxt[s] = *reinterpret_cast<const float4*>(sp + (long long)s * g.total + go);
    }
    int go, lo;
    IO::coords(g, 0, q, go, lo);
    const int line = go / n, j = go - line * n;
    double wl = 1.0;
    if (a.neumann) {
      const int gl = line0 + line;
      const int y = gl % n1, z = three ? gl / n1 : 0;
      if (y == 0 || y == n1 - 1) wl *= 0.5;
      if (three && (z == 0 || z == n2 - 1)) wl *= 0.5;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      float u[NS], gg[NS], o[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        u[s] = vget<float>(cur[s], e);
        gg[s] = buf[lo + s * n * IO::P + e * IO::P];
      }
      const double w = a.neumann && (j + e == 0 || j + e == n - 1) ? 0.5 * wl : wl;
      rxn_adjoint<float, NS>(a.rxn, u, gg, o, w, pacc, want_p);
#pragma unroll
      for (int s = 0; s < NS; ++s) buf[lo + s * n * IO::P + e * IO::P] = o[s];
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) cur[s] = nxt[s];
  }
}

// Forward reaction on an x tile in the XTileIO layout: each thread takes 4
// consecutive points of a line (all species) per vector, with every LDS read
// of a vector issued before its arithmetic (conflict-free, as the tile
// commit). The same per-point arithmetic as pw_reaction_n; the stage values
// are stored for the adjoint by the caller.
template <int NS, int KIND>
__device__ __forceinline__ bool x_reaction_vec(const StageArgs<float>& a, float* buf) {
  using IO = XTileIO<32>;
  const Geom& g = a.g;
  const RxnT<float> rx(a.rxn);
  const int n = g.n;
  const int nv = 1 << IO::vshift(g);  // vectors per species, a multiple of 512
  bool bad = false;
#pragma unroll 1
  for (int q = threadIdx.x; q < nv; q += 512) {
    int go, lo;
    IO::coords(g, 0, q, go, lo);
    float u[4][NS];
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int s = 0; s < NS; ++s) u[e][s] = buf[lo + s * n * IO::P + e * IO::P];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      float f[NS];
      rxn_eval_k<float, NS, KIND>(rx, u[e], f);
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        bad |= !isfinite(u[e][s]) || !isfinite(f[s]);
        buf[lo + s * n * IO::P + e * IO::P] = f[s];
      }
    }
  }
  return bad;
}

// Forward reaction of the FAST x kernels: the vector path for one or two
// species without a manufactured source, else the generic pass.
__device__ __forceinline__ bool x_reaction_fast(const StageArgs<float>& a, float* buf,
                                                long long tile) {
  // the kind is uniform: one loop per kind, no branch inside it
  if (a.S == 2) {
    switch (a.rxn.kind) {
      case RXN_LINEAR: return x_reaction_vec<2, RXN_LINEAR>(a, buf);
      case RXN_FHN: return x_reaction_vec<2, RXN_FHN>(a, buf);
      case RXN_GRAY_SCOTT: return x_reaction_vec<2, RXN_GRAY_SCOTT>(a, buf);
      case RXN_SCHNAKENBERG: return x_reaction_vec<2, RXN_SCHNAKENBERG>(a, buf);
      case RXN_GM: return x_reaction_vec<2, RXN_GM>(a, buf);
      default: break;
    }
  }
  if (a.S == 1 && a.rxn.kind == RXN_LINEAR) return x_reaction_vec<1, RXN_LINEAR>(a, buf);
  return pw_reaction(a, buf, tile, false);
}

// The reaction of the register-fed x kernels: kind RK when the launch fixes
// it (RK >= 0), else chosen at run time.
template <int RK>
__device__ __forceinline__ bool x_reaction_sel(const StageArgs<float>& a, float* buf,
                                               long long tile) {
  if constexpr (RK >= 0)
    return x_reaction_vec<2, RK>(a, buf);
  else
    return x_reaction_fast(a, buf, tile);
}

__device__ __forceinline__ void xadj_reaction_fast(const StageArgs<float>& a, float* buf,
                                                   long long tile, double* pacc) {
  switch (a.S) {
    case 1: xadj_reaction_vec<1>(a, buf, tile, pacc); break;
    case 2: xadj_reaction_vec<2>(a, buf, tile, pacc); break;
    default: pw_adj_reaction(a, buf, tile, pacc); break;
  }
}

// FP64 tiles (W = 16 lines, 512 threads) moved through registers, CAP
// vectors of two doubles per thread, when the launch allows it (g.fast, set
// by the host for full tiles of at most two species, 16-byte aligned fields,
// n a multiple of 64 up to 256 on strided axes and n = 64, 128 or 256 on the
// x axis) and the tile needs at most CAP vectors:
//   strided axes: thread t moves columns 2(t%8), +1 of rows t/8 + 64k;
//   x axis: consecutive threads move consecutive point pairs of a line.
template <int CAP>
struct TileIOF64 {
  double2 v[CAP];
  // vectors per thread: n/64 per species in both layouts
  __device__ __forceinline__ static int nvec(const Geom& g) { return g.spt * (g.n >> 6); }
  __device__ __forceinline__ static bool usable(const Geom& g) {
    return g.fast && nvec(g) <= CAP;
  }
  // Vector m = s (n/64) + k of this thread (species s, block k) sits at
  //   global  tile base + s total + gb + k gk,   LDS  s n pitch + lb + k lk:
  // x tiles are contiguous per species (pair q = t + 512k at offset 2q, tile
  // row 2(q mod n/2), column q / (n/2)); strided rows are t/8 + 64k.
  struct Map {
    long long gb, gk;
    int lb, lk, ps, per;
  };
  __device__ __forceinline__ static Map map(const Geom& g) {
    Map mp;
    const int t = (int)threadIdx.x;
    mp.per = g.n >> 6;
    if (g.inner == 1) {
      const int half = g.n >> 1;
      mp.gb = 2 * t;
      mp.gk = 1024;
      mp.lb = 2 * (t & (half - 1)) * g.pitch + t / half;
      mp.lk = 1024 / g.n;
      mp.ps = g.pitch;  // the pair's two points are consecutive rows
    } else {
      mp.gb = (long long)(t >> 3) * g.inner + 2 * (t & 7);
      mp.gk = 64 * g.inner;
      mp.lb = (t >> 3) * g.pitch + 2 * (t & 7);
      mp.lk = 64 * g.pitch;
      mp.ps = 1;  // consecutive columns
    }
    return mp;
  }
  __device__ __forceinline__ void issue(const Geom& g, const TileRef& tr, const double* src) {
    const Map mp = map(g);
    const int nv = nvec(g);
    const double* sp = src + tr.base + mp.gb;
#pragma unroll
    for (int m = 0; m < CAP; ++m) {
      if (m < nv) {
        const int s = m / mp.per, k = m - s * mp.per;
        v[m] = *reinterpret_cast<const double2*>(sp + s * g.total + k * mp.gk);
      }
    }
  }
  __device__ __forceinline__ void commit(const Geom& g, double* buf) const {
    const Map mp = map(g);
    const int nv = nvec(g);
#pragma unroll
    for (int m = 0; m < CAP; ++m) {
      if (m < nv) {
        const int s = m / mp.per, k = m - s * mp.per;
        double* b = buf + s * g.n * g.pitch + mp.lb + k * mp.lk;
        b[0] = v[m].x;
        b[mp.ps] = v[m].y;
      }
    }
  }
  __device__ __forceinline__ static void store(const Geom& g, const TileRef& tr, const double* buf,
                                               double* dst) {
    const Map mp = map(g);
    const int nv = nvec(g);
    double* dp = dst + tr.base + mp.gb;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      if (m < nv) {
        const int s = m / mp.per, k = m - s * mp.per;
        const double* b = buf + s * g.n * g.pitch + mp.lb + k * mp.lk;
        *reinterpret_cast<double2*>(dp + s * g.total + k * mp.gk) = make_double2(b[0], b[mp.ps]);
      }
    }
  }
};

// Register prefetch of a tile. FAST FP32 kernels (chosen by the host when
// every tile is full, the shapes fit the layouts above and the pointers are
// 16-byte aligned) move tiles with TileIO only; the other FP32 kernels with
// the generic paths, loading in place. Keeping the two apart keeps the
// compiler's wait counts exact on the fast path. FP64 kernels decide per
// launch (the specialisation below).
template <typename T, int W, bool FAST, bool XAX>
struct TilePipe {
  using IO = typename std::conditional<XAX && std::is_same<T, float>::value, XTileIO<W>,
                                       TileIO<T, W>>::type;
  float4 v[XAX ? W / 4 : 4];
  // Past the last tile the last one is loaded again (unused), so that every
  // iteration issues the same loads and the compiler's wait counts stay exact.
  __device__ __forceinline__ void issue(const Geom& g, long long tile, const T* src) {
    if (FAST) IO::issue(g, tile_ref(g, tile < g.ntiles ? tile : g.ntiles - 1), src, v);
  }
  __device__ __forceinline__ void commit(const Geom& g, long long tile, const T* src, T* buf) {
    if (FAST)
      IO::commit(g, v, buf);
    else
      load_tile_fast(g, tile, src, buf, g.spt);
  }
};

// FP64 matrix-core tiles: the next tile in registers where TileIOF64 applies
// (x-axis kernels hold up to 8 vectors per thread, the others 4), else the
// generic in-place loads.
template <bool XAX>
struct TilePipe<double, 16, false, XAX> {
  using IO = TileIOF64<XAX ? 8 : 4>;
  IO io;
  __device__ __forceinline__ void issue(const Geom& g, long long tile, const double* src) {
    if (IO::usable(g)) io.issue(g, tile_ref(g, tile < g.ntiles ? tile : g.ntiles - 1), src);
  }
  __device__ __forceinline__ void commit(const Geom& g, long long tile, const double* src,
                                         double* buf) {
    if (IO::usable(g))
      io.commit(g, buf);
    else
      load_tile_fast(g, tile, src, buf, g.spt);
  }
};

template <typename T, int W, bool FAST, bool XAX>
__device__ __forceinline__ void tile_store(const Geom& g, long long tile, const T* buf, T* dst) {
  using IO = typename std::conditional<XAX && std::is_same<T, float>::value, XTileIO<W>,
                                       TileIO<T, W>>::type;
  if constexpr (std::is_same<T, double>::value && !FAST) {
    if (g.fast && TileIOF64<8>::nvec(g) <= 8) {
      TileIOF64<8>::store(g, tile_ref(g, tile), buf, dst);
      return;
    }
  }
  if (FAST)
    IO::store(g, tile_ref(g, tile), buf, dst);
  else
    store_tile_fast(g, tile, buf, dst, g.spt);
}

// Arrays a forward stage reads for one strided FP32 tile of n = 64, 128 or
// 256 rows, loaded one tile ahead in the thread layout of TileIO<float, 32>
// (straight-line loads: row blocks past n load block 0 again, unused):
//   r1, r2 = stage 0: u_hat, -;  1: u_hat, acc;  2: acc, c_tilde;  3: acc, -
// and L when the plan reads an L table.
template <int MODE>
struct StageLoads {
  float4 L[4], r1[4], r2[4];
  __device__ __forceinline__ void issue(const StageArgs<float>& a, long long tile) {
    using IO = TileIO<float, 32>;
    const TileRef tr = tile_ref(a.g, tile);
    const long long inner = a.g.inner;
    const long long i0 = tr.base + IO::row0() * inner + IO::lane4();
    const float* p1 = MODE <= 1 ? a.uhat : a.acc;
    const float* p2 = MODE == 1 ? a.acc : a.ctil;
#pragma unroll
    for (int k = 0; k < IO::MAXK; ++k) {
      const long long i = i0 + (64 * k < a.g.n ? k : 0) * IO::RSTEP * inner;
      if (!a.lfly) L[k] = *reinterpret_cast<const float4*>(a.ltab + i);
      r1[k] = *reinterpret_cast<const float4*>(p1 + i);
      if (MODE == 1 || MODE == 2) r2[k] = *reinterpret_cast<const float4*>(p2 + i);
    }
  }
};

// Stage combine of one strided FP32 tile (64, 128 or 256 rows) from
// preloaded arrays (same arithmetic as combine_vec). With a.lfly, L = kt_s Lambda^ha_s is formed
// from the eigenvalue tables in LDS ([n0] x, [n1] y, then the transformed
// last axis); the last axis has one outer block per species.
template <int MODE>
__device__ __forceinline__ void combine_pre(const StageArgs<float>& a, float* buf, long long tile,
                                            const StageLoads<MODE>& ld, const float* lam_lds) {
  using IO = TileIO<float, 32>;
  const Geom& g = a.g;
  const TileRef tr = tile_ref(g, tile);
  const long long cst = (long long)a.S * g.total;
  const int r0 = IO::row0(), w4 = IO::lane4();
  const long long inner = g.inner;
  const long long i0 = tr.base + r0 * inner + w4;
  const float cs = a.cs, tau = a.tau;
  float lxy[4], kt = 0.f, ha = 0.f;
  const float* lz = lam_lds;
  if (a.lfly) {
    long long o, rt;
    split_tile(g, tile, o, rt);
    const int s = (int)o;
    const int ib = (int)rt * 32 + w4;
    const int n0 = (int)a.n0, n1 = (int)a.n1;
    const bool three = a.n2 > 1;
    lz = lam_lds + n0 + (three ? n1 : 0);
    // the four lanes of a vector share y (n0 is a multiple of 4)
    const int y = three ? ib / n0 : 0;
    const float* lx = lam_lds + (three ? ib - y * n0 : ib);
    const float ly = three ? lam_lds[n0 + y] : 0.f;
#pragma unroll
    for (int e = 0; e < 4; ++e) lxy[e] = lx[e] + ly;
    kt = pick_species(a.kt, s);
    ha = pick_species(a.ha, s);
  }
#pragma unroll
  for (int k = 0; k < IO::MAXK; ++k) {
    if (64 * k >= g.n) break;
    const long long i = i0 + k * IO::RSTEP * inner;
    float* cell = buf + (r0 + IO::RSTEP * k) * IO::P + w4;
    const float4 fh = make_float4(cell[0], cell[1], cell[2], cell[3]);
    const float lr = a.lfly ? lz[r0 + IO::RSTEP * k] : 0.f;
    float4 o0, o1, out;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      float L;
      if (a.lfly) {
        // Lambda >= the smallest nonzero eigenvalue, far from denormals: the
        // hardware log2 / exp2 (about 1 ulp) suffice
        const float lam = lxy[e] + lr;
        L = lam > 0.f ? kt * __builtin_amdgcn_exp2f(ha * __builtin_amdgcn_logf(lam)) : 0.f;
      } else {
        L = vget<float>(ld.L[k], e);
      }
      float c0 = 0.f, c1 = 0.f, c2 = 0.f, c3 = 0.f;
      stage_coefs_L<float>(MODE, L, tau, c0, c1, c2, c3);
      const float f = vget<float>(fh, e);
      const float x1 = vget<float>(ld.r1[k], e);
      if (MODE == 0) {
        const float av = dec_mul(c0, x1) + c1 * f;
        vset<float>(o0, e, dec_mul(c0, av) - c1 * f);
        vset<float>(o1, e, dec_mul(c2, x1) + c3 * f);
        vset<float>(out, e, cs * av);
      } else if (MODE == 1) {
        vset<float>(out, e, cs * (dec_mul(c0, x1) + c1 * f));
        vset<float>(o1, e, vget<float>(ld.r2[k], e) + c2 * f);
      } else if (MODE == 2) {
        vset<float>(out, e, cs * (vget<float>(ld.r2[k], e) + 2.f * c1 * f));
        vset<float>(o1, e, x1 + c2 * f);
      } else {
        const float un = x1 + c2 * f;
        vset<float>(o0, e, un);
        vset<float>(out, e, cs * un);
      }
    }
    if (MODE == 0) {
      if (a.st_uhat) *reinterpret_cast<float4*>(a.st_uhat + i) = ld.r1[k];
      *reinterpret_cast<float4*>(a.ctil + i) = o0;
    }
    if (a.st_fhat) *reinterpret_cast<float4*>(a.st_fhat + MODE * cst + i) = fh;
    if (MODE <= 2) *reinterpret_cast<float4*>(a.acc + i) = o1;
    if (MODE == 3) *reinterpret_cast<float4*>(a.uhat + i) = o0;
    cell[0] = out.x;
    cell[1] = out.y;
    cell[2] = out.z;
    cell[3] = out.w;
  }
}

// All six P13 coefficients of L (order C_R, C_Q, C_PHI, C_PHI1, C_PHI2,
// C_PHI3) and, for the parameter gradients, their derivatives in L from the
// quotient rule, g' = (num' - g den') / den, with D' = 18 + 12L + 3L^2 and
// Dh' = 72 + 24L + 3L^2 (Section 4's rational forms).
__device__ __forceinline__ void p13_all(float L, float tau, float* c) {
  const float D = 24.f + L * (18.f + L * (6.f + L));
  const float Dh = 192.f + L * (72.f + L * (12.f + L));
  const float iD = __builtin_amdgcn_rcpf(D), iDh = __builtin_amdgcn_rcpf(Dh);
  const bool small = L < 1.f;
  const float ph = 96.f + L * (12.f + L);
  c[C_R] = small ? 1.f - L * (24.f + L * (6.f + L)) * iD : (24.f - 6.f * L) * iD;
  c[C_Q] = small ? 1.f - L * ph * iDh : 24.f * (8.f - L) * iDh;
  c[C_PHI] = tau * ph * iDh;
  c[C_PHI1] = tau * (4.f - L) * iD;
  c[C_PHI2] = 2.f * tau * (4.f + L) * iD;
  c[C_PHI3] = tau * (4.f + L * (3.f + L)) * iD;
}
__device__ __forceinline__ void p13_dall(float L, float tau, const float* c, float* d) {
  const float D = 24.f + L * (18.f + L * (6.f + L));
  const float Dh = 192.f + L * (72.f + L * (12.f + L));
  const float iD = __builtin_amdgcn_rcpf(D), iDh = __builtin_amdgcn_rcpf(Dh);
  const float dD = 18.f + L * (12.f + 3.f * L), dDh = 72.f + L * (24.f + 3.f * L);
  d[C_R] = (-6.f - c[C_R] * dD) * iD;
  d[C_Q] = (-24.f - c[C_Q] * dDh) * iDh;
  d[C_PHI] = (tau * (12.f + 2.f * L) - c[C_PHI] * dDh) * iDh;
  d[C_PHI1] = (-tau - c[C_PHI1] * dD) * iD;
  d[C_PHI2] = (2.f * tau - c[C_PHI2] * dD) * iD;
  d[C_PHI3] = (tau * (3.f + 2.f * L) - c[C_PHI3] * dD) * iD;
}

// Adjoint combine (same arithmetic as pw_adj_combine, MODE 0..3 or
// MODE_INIT) on a one-species strided FP32 tile, L formed from the LDS
// eigenvalue tables. With TH, each coefficient application's
// y g'(L) x (the G increment) is turned into the kappa and alpha gradient
// contributions at once: times the spectral weight, then by dL/dkappa =
// tau Lambda^(alpha/2) and dL/dalpha = L ln(Lambda) / 2, summed per thread
// and tile in FP32 and across tiles in FP64 (acc[2s], acc[2s + 1]).
// Adjoint stage arrays loaded ahead of the forward transform (up to four per
// stage, in the thread layout of TileIO<float, 32>):
//   0: z, [u_hat, f_u, f_a];  1: z, aacc, [u_hat, f_a];  2: a_hat, aacc, gu, [u_hat];
//   3: aacc;  MODE_INIT: none  (bracketed: with the kappa/alpha gradients).
template <int MODE, bool TH>
struct AdjLoads {
  static constexpr int NQ = MODE == 0 ? (TH ? 4 : 1)
                          : MODE == 1 ? (TH ? 4 : 2)
                          : MODE == 2 ? (TH ? 4 : 3)
                          : MODE == 3 ? 1 : 0;
  float4 q[NQ > 0 ? NQ : 1][4];
  __device__ __forceinline__ static const float* src(const StageArgs<float>& a, int j) {
    const long long cst = (long long)a.S * a.g.total;
    if (MODE == 0) return j == 0 ? a.zh : j == 1 ? a.st_uhat : j == 2 ? a.st_fhat : a.st_fhat + cst;
    if (MODE == 1) return j == 0 ? a.zh : j == 1 ? a.aacc : j == 2 ? a.st_uhat : a.st_fhat + cst;
    if (MODE == 2) return j == 0 ? a.ahat : j == 1 ? a.aacc : j == 2 ? a.gu : a.st_uhat;
    return a.aacc;
  }
  // arrays j0 .. j1-1
  template <int J0 = 0, int J1 = NQ>
  __device__ __forceinline__ void issue(const StageArgs<float>& a, long long tile) {
    using IO = TileIO<float, 32>;
    const TileRef tr = tile_ref(a.g, tile);
    const long long inner = a.g.inner;
    const long long i0 = tr.base + IO::row0() * inner + IO::lane4();
#pragma unroll
    for (int j = J0; j < (J1 < NQ ? J1 : NQ); ++j) {
      const float* p = src(a, j);
#pragma unroll
      for (int k = 0; k < IO::MAXK; ++k)
        q[j][k] = *reinterpret_cast<const float4*>(p + i0 + (64 * k < a.g.n ? k : 0) * IO::RSTEP * inner);
    }
  }
};

template <int MODE, bool TH, bool PRE = false>
__device__ __forceinline__ void zadj_tile32(const StageArgs<float>& a, float* buf, long long tile,
                                            const float* lam_lds, double (&acc)[4],
                                            const AdjLoads<MODE, TH>* ld = nullptr) {
  using IO = TileIO<float, 32>;
  const Geom& g = a.g;
  const TileRef tr = tile_ref(g, tile);
  const long long cst = (long long)a.S * g.total;
  const int r0 = IO::row0(), w4 = IO::lane4();
  const long long inner = g.inner;
  const long long i0 = tr.base + r0 * inner + w4;
  const float cs = a.cs, tau = a.tau;
  long long o, rt;
  split_tile(g, tile, o, rt);
  const int s = (int)o;
  const int ib = (int)rt * 32 + w4;
  const int n0 = (int)a.n0, n1 = (int)a.n1;
  const bool three = a.n2 > 1;
  const float* lz = lam_lds + n0 + (three ? n1 : 0);
  const int y = three ? ib / n0 : 0;
  const int x0 = three ? ib - y * n0 : ib;
  const float* lx = lam_lds + x0;
  const float ly = three ? lam_lds[n0 + y] : 0.f;
  // spectral weights: cs times the Neumann end weights
  float wxy[4];
  {
    const bool neu = a.neumann;
    const float wy = (neu && three && (y == 0 || y == n1 - 1)) ? 0.5f : 1.f;
#pragma unroll
    for (int e = 0; e < 4; ++e)
      wxy[e] = cs * wy * ((neu && (x0 + e == 0 || x0 + e == n0 - 1)) ? 0.5f : 1.f);
  }
  const float kt = pick_species(a.kt, s), ha = pick_species(a.ha, s);
  // per-tile sums in FP32 (at most 16 terms per thread), added in FP64
  float acc_k = 0.f, acc_a = 0.f;
#pragma unroll
  for (int k = 0; k < IO::MAXK; ++k) {
    if (64 * k >= g.n) break;
    const int row = r0 + IO::RSTEP * k;
    const long long i = i0 + k * IO::RSTEP * inner;
    float* cell = buf + row * IO::P + w4;
    const float4 Xv = make_float4(cell[0], cell[1], cell[2], cell[3]);
    float4 z4, a4, h4, u4, gu4, f0, f1, f2, f3;
    if constexpr (PRE) {
      if (MODE == 0) {
        z4 = ld->q[0][k];
        if (TH) {
          u4 = ld->q[TH ? 1 : 0][k];
          f0 = ld->q[TH ? 2 : 0][k];
          f1 = ld->q[TH ? 3 : 0][k];
          f2 = *reinterpret_cast<const float4*>(a.st_fhat + 2 * cst + i);
          f3 = *reinterpret_cast<const float4*>(a.st_fhat + 3 * cst + i);
        }
      } else if (MODE == 1) {
        z4 = ld->q[0][k];
        a4 = ld->q[1][k];
        if (TH) {
          u4 = ld->q[TH ? 2 : 0][k];
          f1 = ld->q[TH ? 3 : 0][k];
        }
      } else if (MODE == 2) {
        h4 = ld->q[0][k];
        a4 = ld->q[1][k];
        gu4 = ld->q[2][k];
        if (TH) {
          u4 = ld->q[TH ? 3 : 0][k];
          f0 = *reinterpret_cast<const float4*>(a.st_fhat + i);
        }
      } else if (MODE == 3) {
        a4 = ld->q[0][k];
      }
    } else {
    if (MODE == 0 || MODE == 1) z4 = *reinterpret_cast<const float4*>(a.zh + i);
    if (MODE == 1 || MODE == 2 || MODE == 3) a4 = *reinterpret_cast<const float4*>(a.aacc + i);
    if (MODE == 2) {
      h4 = *reinterpret_cast<const float4*>(a.ahat + i);
      gu4 = *reinterpret_cast<const float4*>(a.gu + i);
    }
    if (TH && MODE <= 2) {
      u4 = *reinterpret_cast<const float4*>(a.st_uhat + i);
      if (MODE == 0 || MODE == 2) f0 = *reinterpret_cast<const float4*>(a.st_fhat + i);
      if (MODE == 0 || MODE == 1) f1 = *reinterpret_cast<const float4*>(a.st_fhat + cst + i);
      if (MODE == 0) {
        f2 = *reinterpret_cast<const float4*>(a.st_fhat + 2 * cst + i);
        f3 = *reinterpret_cast<const float4*>(a.st_fhat + 3 * cst + i);
      }
    }
    }
    const float lr = lz[row];
    const float wz = (a.neumann && (row == 0 || row == g.n - 1)) ? 0.5f : 1.f;
    float4 out, o1, o2, o3;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float lam = lx[e] + ly + lr;
      const float lg = lam > 0.f ? __builtin_amdgcn_logf(lam) : 0.f;  // log2(Lambda)
      const float pw = lam > 0.f ? __builtin_amdgcn_exp2f(ha * lg) : 0.f;
      const float L = kt * pw;
      float c[NCOEF];
      p13_all(L, tau, c);
      const float X = vget<float>(Xv, e);
      float ov = 0.f, gsum = 0.f;
      if (MODE == 0) {
        const float z = vget<float>(z4, e);
        vset<float>(o1, e, c[C_R] * z);
        vset<float>(o2, e, c[C_Q] * X);
        vset<float>(o3, e, c[C_PHI1] * z - c[C_PHI] * X);
        ov = c[C_PHI2] * z + 2.f * c[C_PHI] * X;
        if (TH) {
          float d[NCOEF];
          p13_dall(L, tau, c, d);
          const float uh = vget<float>(u4, e), fu = vget<float>(f0, e), fa = vget<float>(f1, e);
          const float fb = vget<float>(f2, e), fc = vget<float>(f3, e);
          const float ah = c[C_Q] * uh + c[C_PHI] * fu;
          const float s1 = d[C_R] * uh + d[C_PHI1] * fu + d[C_PHI2] * (fa + fb) + d[C_PHI3] * fc;
          const float s2 = d[C_Q] * ah + d[C_PHI] * (2.f * fb - fu);
          gsum = z * s1 + X * s2;
        }
      } else if (MODE == 1) {
        const float z = vget<float>(z4, e);
        vset<float>(o1, e, vget<float>(a4, e) + c[C_Q] * X);
        ov = c[C_PHI2] * z + c[C_PHI] * X;
        if (TH) {
          float d[NCOEF];
          p13_dall(L, tau, c, d);
          gsum = X * (d[C_Q] * vget<float>(u4, e) + d[C_PHI] * vget<float>(f1, e));
        }
      } else if (MODE == 2) {
        const float A = vget<float>(h4, e) + X;
        vset<float>(o1, e, vget<float>(a4, e) + c[C_Q] * A);
        ov = vget<float>(gu4, e) + c[C_PHI] * A;
        if (TH) {
          float d[NCOEF];
          p13_dall(L, tau, c, d);
          gsum = A * (d[C_Q] * vget<float>(u4, e) + d[C_PHI] * vget<float>(f0, e));
        }
      } else if (MODE == 3) {
        const float zn = vget<float>(a4, e) + X;
        vset<float>(o1, e, zn);
        ov = a.last ? zn : c[C_PHI3] * zn;
      } else {  // MODE_INIT
        vset<float>(o1, e, X);
        ov = c[C_PHI3] * X;
      }
      vset<float>(out, e, cs * ov);
      if (TH && MODE <= 2 && lam > 0.f) {
        const float gw = wxy[e] * wz * gsum;
        acc_k += gw * (tau * pw);
        acc_a += gw * (0.34657359f * L * lg);  // L ln(Lambda) / 2
      }
    }
    if (MODE == 0) {
      *reinterpret_cast<float4*>(a.aacc + i) = o1;
      *reinterpret_cast<float4*>(a.ahat + i) = o2;
      *reinterpret_cast<float4*>(a.gu + i) = o3;
    } else if (MODE == 1 || MODE == 2) {
      *reinterpret_cast<float4*>(a.aacc + i) = o1;
    } else {
      *reinterpret_cast<float4*>(a.zh + i) = o1;
    }
    cell[0] = out.x;
    cell[1] = out.y;
    cell[2] = out.z;
    cell[3] = out.w;
  }
  if (TH) {
    if (s == 0) {
      acc[0] += double(acc_k);
      acc[1] += double(acc_a);
    } else {
      acc[2] += double(acc_k);
      acc[3] += double(acc_a);
    }
  }
}

template <bool TH>
__device__ __forceinline__ void zadj_vec(const StageArgs<float>& a, float* buf, long long tile,
                                         const float* lam_lds, double (&acc)[4]) {
  switch (a.mode) {
    case 0: zadj_tile32<0, TH>(a, buf, tile, lam_lds, acc); break;
    case 1: zadj_tile32<1, TH>(a, buf, tile, lam_lds, acc); break;
    case 2: zadj_tile32<2, TH>(a, buf, tile, lam_lds, acc); break;
    case 3: zadj_tile32<3, false>(a, buf, tile, lam_lds, acc); break;
    default: zadj_tile32<MODE_INIT, false>(a, buf, tile, lam_lds, acc); break;
  }
}

// Forward stage combine on a one-species strided FP32 tile, in the thread
// layout of TileIO<float, 32> (same arithmetic as combine_vec).
template <int MODE, bool LT>
__device__ __forceinline__ void combine_tile32(const StageArgs<float>& a, float* buf,
                                               const TileRef& tr) {
  using IO = TileIO<float, 32>;
  const Geom& g = a.g;
  const long long cst = (long long)a.S * g.total;
  const int r0 = IO::row0(), w4 = IO::lane4();
  const long long inner = g.inner;
  const long long i0 = tr.base + r0 * inner + w4;
  const float cs = a.cs, tau = a.tau;
#pragma unroll 1
  for (int k = 0; k < IO::MAXK; ++k) {
    if (64 * k >= g.n) break;
    const long long i = i0 + k * IO::RSTEP * inner;
    float* cell = buf + (r0 + IO::RSTEP * k) * IO::P + w4;
    float4 Lv, t0, t1, t2, t3, uh, ac, ct;
    if (LT) {
      Lv = *reinterpret_cast<const float4*>(a.ltab + i);
    } else {
      const float* cf = a.coef + i;
      if (MODE <= 1) t0 = *reinterpret_cast<const float4*>(cf + C_Q * cst);
      if (MODE <= 2) t1 = *reinterpret_cast<const float4*>(cf + C_PHI * cst);
      t2 = *reinterpret_cast<const float4*>(
          cf + (MODE == 0 ? C_R : MODE == 3 ? C_PHI3 : C_PHI2) * cst);
      if (MODE == 0) t3 = *reinterpret_cast<const float4*>(cf + C_PHI1 * cst);
    }
    if (MODE <= 1) uh = *reinterpret_cast<const float4*>(a.uhat + i);
    if (MODE >= 1) ac = *reinterpret_cast<const float4*>(a.acc + i);
    if (MODE == 2) ct = *reinterpret_cast<const float4*>(a.ctil + i);
    float4 fh = make_float4(cell[0], cell[1], cell[2], cell[3]);
    float4 o0, o1, out;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      float c0 = 0.f, c1 = 0.f, c2 = 0.f, c3 = 0.f;
      if (LT) {
        stage_coefs_L<float>(MODE, vget<float>(Lv, e), tau, c0, c1, c2, c3);
      } else {
        if (MODE <= 1) c0 = vget<float>(t0, e);
        if (MODE <= 2) c1 = vget<float>(t1, e);
        c2 = vget<float>(t2, e);
        if (MODE == 0) c3 = vget<float>(t3, e);
      }
      const float f = vget<float>(fh, e);
      if (MODE == 0) {
        const float u = vget<float>(uh, e);
        const float av = dec_mul(c0, u) + c1 * f;
        vset<float>(o0, e, dec_mul(c0, av) - c1 * f);
        vset<float>(o1, e, dec_mul(c2, u) + c3 * f);
        vset<float>(out, e, cs * av);
      } else if (MODE == 1) {
        vset<float>(out, e, cs * (dec_mul(c0, vget<float>(uh, e)) + c1 * f));
        vset<float>(o1, e, vget<float>(ac, e) + c2 * f);
      } else if (MODE == 2) {
        vset<float>(out, e, cs * (vget<float>(ct, e) + 2.f * c1 * f));
        vset<float>(o1, e, vget<float>(ac, e) + c2 * f);
      } else {
        const float un = vget<float>(ac, e) + c2 * f;
        vset<float>(o0, e, un);
        vset<float>(out, e, cs * un);
      }
    }
    if (MODE == 0) {
      if (a.st_uhat) *reinterpret_cast<float4*>(a.st_uhat + i) = uh;
      *reinterpret_cast<float4*>(a.ctil + i) = o0;
    }
    if (a.st_fhat) *reinterpret_cast<float4*>(a.st_fhat + MODE * cst + i) = fh;
    if (MODE <= 2) *reinterpret_cast<float4*>(a.acc + i) = o1;
    if (MODE == 3) *reinterpret_cast<float4*>(a.uhat + i) = o0;
    cell[0] = out.x;
    cell[1] = out.y;
    cell[2] = out.z;
    cell[3] = out.w;
  }
}

template <typename T, int W, bool FAST>
__device__ __forceinline__ void combine_tile(const StageArgs<T>& a, T* buf, long long tile) {
  if constexpr (FAST && std::is_same<T, float>::value && W == 32) {
    const TileRef tr = tile_ref(a.g, tile);
    if (a.mode <= 3 && a.g.spt == 1) {
      const bool lt = a.ltab != nullptr;
      switch (a.mode) {
        case 0:
          lt ? combine_tile32<0, true>(a, buf, tr) : combine_tile32<0, false>(a, buf, tr);
          return;
        case 1:
          lt ? combine_tile32<1, true>(a, buf, tr) : combine_tile32<1, false>(a, buf, tr);
          return;
        case 2:
          lt ? combine_tile32<2, true>(a, buf, tr) : combine_tile32<2, false>(a, buf, tr);
          return;
        default:
          lt ? combine_tile32<3, true>(a, buf, tr) : combine_tile32<3, false>(a, buf, tr);
          return;
      }
    }
  }
  pw_combine_fast(a, buf, tile);
}

// Forward combine of one stage known at compile time (the FP64 per-stage Z
// kernels): vectors on full strided tiles, else the generic pass.
template <typename T, int MODE>
__device__ __forceinline__ void combine_mode(const StageArgs<T>& a, T* buf, long long tile) {
  const TileRef tr = tile_ref(a.g, tile);
  if (a.g.inner == 1 || !tile_vectorizable<T>(a.g, tr, a.uhat)) {
    pw_combine(a, buf, tile);
    return;
  }
  if (a.ltab)
    combine_vec<T, MODE, true>(a, buf, tr);
  else
    combine_vec<T, MODE, false>(a, buf, tr);
}

// Inputs of the fold of an x tile (two species, 32 lines, n in {64, 128,
// 256}, DCT-I / DST-I), read straight into registers: thread t takes line
// (t/16) mod 32, entries i0 .. i0+7 and n-8-i0 .. n-1-i0 with i0 = 8 (t%16)
// (padding items, i0 >= n/2, read entry 0 again and are dropped). Where
// i0 >= 64 the two float4 of each group come in swapped order: the fold
// buffer's rotated entries (MfmaXfF32::fold).
struct XFoldLoads {
  float4 v[2][4];
  __device__ __forceinline__ void issue(const Geom& g, long long tile, const float* src) {
    const long long t = tile < g.ntiles ? tile : g.ntiles - 1;
    const int n = g.n;
    const int i0 = (threadIdx.x & 15) << 3;
    const int ic = 2 * i0 < n ? i0 : 0;
    const int sw = (threadIdx.x & 8) ? 4 : 0;  // i0 >= 64
    const long long line = t * 32 + ((threadIdx.x >> 4) & 31);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const float* p = src + s * g.total + line * n;
      v[s][0] = *reinterpret_cast<const float4*>(p + ic + sw);
      v[s][1] = *reinterpret_cast<const float4*>(p + ic + 4 - sw);
      v[s][2] = *reinterpret_cast<const float4*>(p + n - 8 - ic + sw);
      v[s][3] = *reinterpret_cast<const float4*>(p + n - 4 - ic - sw);
    }
  }
};

// ------------------------------------------------------------------ kernels
// Persistent: block b handles tiles b, b + gridDim.x, ... The loads of the
// next tile are issued before the current one is computed and written to LDS
// after its stores: the wait then covers those loads only (the stores just
// issued stay in flight), on the one path through the loop body. Past the
// last tile, the last one is loaded again and dropped.
// RK >= 0 (FAST FP32, two species, non-periodic x axis: the host checks):
// only the register-fed path with reaction kind RK is compiled. A kernel
// holding every path and kind is several times the size of the instruction
// cache, and each launch then waits on instruction fetches.
template <typename T, class XF, bool FAST, int RK = -1>
__global__ __launch_bounds__(XF::THREADS, XF::MIN_WAVES_PER_EU) void k_xstage_m(StageArgs<T> a, MfmaAxisDev ax) {
  to_member(a);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* buf = reinterpret_cast<T*>(smem_raw);
  XF xf(&a.g, &ax, reinterpret_cast<T*>(smem_raw + ax.fb_off));
  const int S = a.g.spt;
  const int last = (int)(a.g.ntiles - 1);
  bool bad = false;
  if constexpr (FAST && std::is_same<T, float>::value) {
    if (RK >= 0 || (ax.direct && S == 2)) {
      // inverse-x folded straight from registers: no LDS staging of the input
      XFoldLoads rl;
      rl.issue(a.g, blockIdx.x, a.P);
      for (int tile = blockIdx.x; tile < a.g.ntiles; tile += gridDim.x) {
        const int next = tile + gridDim.x < last ? tile + gridDim.x : last;
        xf.fold_regs(rl.v[0]);
        __syncthreads();
        xf.mfma_write(buf, !xf.two_buffers());
        xf.use(1);
        xf.fold_regs(rl.v[1]);
        rl.issue(a.g, next, a.P);
        __syncthreads();
        xf.mfma_write(buf + a.g.n * XF::P);
        xf.use(0);
        if (a.st_phys) {
          XTileIO<XF::W>::store(a.g, tile_ref(a.g, tile), buf,
                                a.st_phys + (long long)a.mode * S * a.g.total);
          __syncthreads();
        }
        bad |= x_reaction_sel<RK>(a, buf, tile);
        __syncthreads();
        xf(buf, S);
        tile_store<T, XF::W, FAST, true>(a.g, tile, buf, a.P);
        __syncthreads();
      }
      if (bad) a.flag[0] = 1;
      return;
    }
  }
  if constexpr (RK >= 0) return;
  TilePipe<T, XF::W, FAST, true> pipe;
  pipe.issue(a.g, blockIdx.x, a.P);
  pipe.commit(a.g, blockIdx.x, a.P, buf);
  __syncthreads();
  for (int tile = blockIdx.x; tile < a.g.ntiles; tile += gridDim.x) {
    const int next = tile + gridDim.x < last ? tile + gridDim.x : last;
    pipe.issue(a.g, next, a.P);
    xf(buf, S);
    if constexpr (FAST && std::is_same<T, float>::value) {
      // stage values stored for the adjoint as vectors of the tile
      if (a.st_phys) {
        XTileIO<XF::W>::store(a.g, tile_ref(a.g, tile), buf,
                              a.st_phys + (long long)a.mode * S * a.g.total);
        __syncthreads();
      }
      bad |= x_reaction_fast(a, buf, tile);
    } else {
      bad |= pw_reaction(a, buf, tile);
    }
    __syncthreads();
    xf(buf, S);
    tile_store<T, XF::W, FAST, true>(a.g, tile, buf, a.P);
    __syncthreads();
    pipe.commit(a.g, next, a.P, buf);
    __syncthreads();
  }
  if (bad) a.flag[0] = 1;
}

// A contiguous run of tiles for this block, [t0, t1), runs balanced over the
// grid (gridDim.x <= ntiles, so no run is empty). With runs instead of a
// stride of gridDim.x, the tiles in flight at one time lie spread over the
// whole field rather than in one slab of it, which the strided rows of a
// last-axis tile read at a higher HBM rate.
struct TileRun {
  int t0, t1;  // the engine launches fewer than 2^31 - 2^16 tiles (host-checked)
  __device__ __forceinline__ explicit TileRun(long long ntiles)
      : t0((int)((long long)blockIdx.x * ntiles / gridDim.x)),
        t1((int)(((long long)blockIdx.x + 1) * ntiles / gridDim.x)) {}
  __device__ __forceinline__ int next(int tile) const { return tile + 1 < t1 ? tile + 1 : t1 - 1; }
};

// MODE >= 0 (FAST FP32 plans, forward stages; last axes of 64, 128, 192 or
// 256 points): the stage arrays of the next tile are loaded while this one is
// computed, each block taking a run of tiles. MODE < 0 takes a.mode at run
// time.
template <typename T, class XF, int MODE, bool FAST>
__global__ __launch_bounds__(XF::THREADS, XF::MIN_WAVES_PER_EU) void k_zstage_m(StageArgs<T> a, MfmaAxisDev ax) {
  to_member(a);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* buf = reinterpret_cast<T*>(smem_raw);
  XF xf(&a.g, &ax, reinterpret_cast<T*>(smem_raw + ax.fb_off));
  const T* src = a.src ? a.src : a.P;
  const int S = a.g.spt;
  TilePipe<T, XF::W, FAST, false> pipe;
  if constexpr (FAST && MODE >= 0 && std::is_same<T, float>::value && XF::W == 32) {
    const TileRun run(a.g.ntiles);
    pipe.issue(a.g, run.t0, src);
    // eigenvalue tables for L formed in the kernel
    float* lam_lds = reinterpret_cast<float*>(smem_raw + a.lam_off);
    if (a.lfly) {
      const int nx = (int)a.n0, ny = (int)a.n1, nz = a.n2 > 1 ? (int)a.n2 : 0;
      for (int i = threadIdx.x; i < nx + ny + nz; i += blockDim.x)
        lam_lds[i] = float(i < nx ? a.lam[0][i]
                                  : (i < nx + ny ? a.lam[1][i - nx] : a.lam[2][i - nx - ny]));
    }
    StageLoads<MODE> ld;
    ld.issue(a, run.t0);
    pipe.commit(a.g, run.t0, src, buf);
    __syncthreads();
    for (int tile = run.t0; tile < run.t1; ++tile) {
      const int next = run.next(tile);
      pipe.issue(a.g, next, src);
      xf(buf, 1);
      combine_pre<MODE>(a, buf, tile, ld, lam_lds);
      ld.issue(a, next);
      __syncthreads();
      if (ax.direct) {
        // inverse transform straight to the field
        xf.to_global(buf, a.P + tile_ref(a.g, tile).base, a.g.inner);
      } else {
        xf(buf, 1);
        tile_store<T, XF::W, FAST, false>(a.g, tile, buf, a.P);
        __syncthreads();
      }
      pipe.commit(a.g, next, src, buf);
      __syncthreads();
    }
  } else {
    const TileRun run(a.g.ntiles);
    pipe.issue(a.g, run.t0, src);
    pipe.commit(a.g, run.t0, src, buf);
    __syncthreads();
    for (int tile = run.t0; tile < run.t1; ++tile) {
      const int next = run.next(tile);
      if (!a.src) xf(buf, S);
      if constexpr (MODE >= 0 && MODE <= 3 && !std::is_same<T, float>::value)
        combine_mode<T, MODE>(a, buf, tile);
      else
        combine_tile<T, XF::W, FAST>(a, buf, tile);
      __syncthreads();
      pipe.issue(a.g, next, src);
      xf(buf, S);
      tile_store<T, XF::W, FAST, false>(a.g, tile, buf, a.P);
      __syncthreads();
      pipe.commit(a.g, next, src, buf);
      __syncthreads();
    }
  }
}

// NS > 0 (FAST FP32 launches of one or two species, chosen by the host): the
// vector adjoint reaction of NS species only. RF (two species, DCT-I /
// DST-I, no reaction-parameter partials): the first transform folded
// straight from registers, as in the forward x kernels (no LDS staging of
// the input tile). KIND >= 0 (FP64, two species, chosen by the host): only
// the adjoint reaction of that kind is compiled (the kernel holding every
// species count and kind is past the size of the instruction cache).
template <typename T, class XF, bool FAST, int NS = 0, bool RF = false, int KIND = -1>
__global__ __launch_bounds__(XF::THREADS, XF::MIN_WAVES_PER_EU) void k_xadj_m(StageArgs<T> a, MfmaAxisDev ax) {
  to_member(a);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* buf = reinterpret_cast<T*>(smem_raw);
  XF xf(&a.g, &ax, reinterpret_cast<T*>(smem_raw + ax.fb_off));
  double pacc[RXN_NP_MAX];
  for (int k = 0; k < RXN_NP_MAX; ++k) pacc[k] = 0.0;
  const int S = a.g.spt;
  const int last = (int)(a.g.ntiles - 1);
  if constexpr (RF && NS == 2 && FAST && std::is_same<T, float>::value && XF::XAX) {
    XFoldLoads rl;
    rl.issue(a.g, blockIdx.x, a.P);
    for (int tile = blockIdx.x; tile < a.g.ntiles; tile += gridDim.x) {
      const int next = tile + gridDim.x < last ? tile + gridDim.x : last;
      xf.fold_regs(rl.v[0]);
      __syncthreads();
      xf.mfma_write(buf, !xf.two_buffers());
      xf.use(1);
      xf.fold_regs(rl.v[1]);
      __syncthreads();
      xf.mfma_write(buf + a.g.n * XF::P);
      xf.use(0);
      xadj_reaction_vec<NS, false>(a, buf, tile, pacc);
      __syncthreads();
      // next tile's input: in flight over the second transform and the store
      // (issued earlier, its registers would be live across the reaction)
      rl.issue(a.g, next, a.P);
      xf(buf, S);
      tile_store<T, XF::W, FAST, true>(a.g, tile, buf, a.P);
      __syncthreads();
    }
    return;
  }
  TilePipe<T, XF::W, FAST, true> pipe;
  pipe.issue(a.g, blockIdx.x, a.P);
  pipe.commit(a.g, blockIdx.x, a.P, buf);
  __syncthreads();
  for (int tile = blockIdx.x; tile < a.g.ntiles; tile += gridDim.x) {
    const int next = tile + gridDim.x < last ? tile + gridDim.x : last;
    xf(buf, S);
    if constexpr (FAST && std::is_same<T, float>::value && XF::XAX && NS > 0)
      xadj_reaction_vec<NS>(a, buf, tile, pacc);
    else if constexpr (FAST && std::is_same<T, float>::value && XF::XAX)
      xadj_reaction_fast(a, buf, tile, pacc);
    else if constexpr (KIND >= 0)
      pw_adj_reaction_n<T, 2, KIND>(a, buf, tile, pacc);
    else
      pw_adj_reaction(a, buf, tile, pacc);
    __syncthreads();
    pipe.issue(a.g, next, a.P);
    xf(buf, S);
    tile_store<T, XF::W, FAST, true>(a.g, tile, buf, a.P);
    __syncthreads();
    pipe.commit(a.g, next, a.P, buf);
    __syncthreads();
  }
  if (a.rp_acc) block_add_partials(reinterpret_cast<double*>(smem_raw), pacc, a.rxn.np, a.rp_acc);
}

// Adjoint Z stage on one-species strided FP32 tiles with L formed in the
// kernel and the stage arrays loaded ahead of the forward transform.
template <class XF, int MODE, bool TH>
__device__ __forceinline__ void zadj_staged(const StageArgs<float>& a, float* buf, XF& xf,
                                            TilePipe<float, XF::W, true, false>& pipe,
                                            const float* lam_lds, double (&acc)[4],
                                            const TileRun& run) {
  AdjLoads<MODE, TH> ld;
  // with the kappa/alpha terms, the stored stage arrays are loaded after the
  // forward transform (fewer registers live across it)
  constexpr int NE = TH ? 2 : AdjLoads<MODE, TH>::NQ;
  for (int tile = run.t0; tile < run.t1; ++tile) {
    const int next = run.next(tile);
    ld.template issue<0, NE>(a, tile);
    xf(buf, 1);
    ld.template issue<NE, AdjLoads<MODE, TH>::NQ>(a, tile);
    zadj_tile32<MODE, TH, true>(a, buf, tile, lam_lds, acc, &ld);
    __syncthreads();
    pipe.issue(a.g, next, a.P);
    xf(buf, 1);
    tile_store<float, XF::W, true, false>(a.g, tile, buf, a.P);
    __syncthreads();
    pipe.commit(a.g, next, a.P, buf);
    __syncthreads();
  }
}

// MODE >= 0: one kernel per adjoint stage (FAST FP32 plans with L formed in
// the kernel); MODE < 0 takes a.mode at run time. THV = 1 / 0 (with MODE >=
// 0): launches with / without the kappa/alpha partials (a.thp), chosen by the
// host where the staged path applies; only that path is compiled.
template <typename T, class XF, bool FAST, int MODE = -1, int THV = -1>
__global__ __launch_bounds__(XF::THREADS, XF::MIN_WAVES_PER_EU) void k_zadj_m(StageArgs<T> a, MfmaAxisDev ax) {
  to_member(a);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* buf = reinterpret_cast<T*>(smem_raw);
  XF xf(&a.g, &ax, reinterpret_cast<T*>(smem_raw + ax.fb_off));
  const int S = a.g.spt;
  const TileRun run(a.g.ntiles);
  TilePipe<T, XF::W, FAST, false> pipe;
  pipe.issue(a.g, run.t0, a.P);
  pipe.commit(a.g, run.t0, a.P, buf);
  if constexpr (FAST && std::is_same<T, float>::value && XF::W == 32) {
    // (a per-point accumulator G, when present, is filled by the generic path)
    if (a.lfly && S == 1 && (a.thp != nullptr || a.G == nullptr)) {
      float* lam_lds = reinterpret_cast<float*>(smem_raw + a.lam_off);
      const int nx = (int)a.n0, ny = (int)a.n1, nz = a.n2 > 1 ? (int)a.n2 : 0;
      for (int i = threadIdx.x; i < nx + ny + nz; i += blockDim.x)
        lam_lds[i] = float(i < nx ? a.lam[0][i]
                                  : (i < nx + ny ? a.lam[1][i - nx] : a.lam[2][i - nx - ny]));
      __syncthreads();
      // kappa, alpha partials of (at most, host-checked) two species
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      const bool th = THV >= 0 ? THV == 1 : a.thp != nullptr;
      if constexpr (MODE >= 0 && THV == 1) {
        zadj_staged<XF, MODE, MODE <= 2>(a, buf, xf, pipe, lam_lds, acc, run);
      } else if constexpr (MODE >= 0 && THV == 0) {
        zadj_staged<XF, MODE, false>(a, buf, xf, pipe, lam_lds, acc, run);
      } else if constexpr (MODE >= 0) {
        if (th)
          zadj_staged<XF, MODE, MODE <= 2>(a, buf, xf, pipe, lam_lds, acc, run);
        else
          zadj_staged<XF, MODE, false>(a, buf, xf, pipe, lam_lds, acc, run);
      } else
      for (int tile = run.t0; tile < run.t1; ++tile) {
        const int next = run.next(tile);
        xf(buf, 1);
        if (th)
          zadj_vec<true>(a, buf, tile, lam_lds, acc);
        else
          zadj_vec<false>(a, buf, tile, lam_lds, acc);
        __syncthreads();
        pipe.issue(a.g, next, a.P);
        xf(buf, 1);
        tile_store<T, XF::W, FAST, false>(a.g, tile, buf, a.P);
        __syncthreads();
        pipe.commit(a.g, next, a.P, buf);
        __syncthreads();
      }
      if (th) block_sums(reinterpret_cast<double*>(smem_raw), acc, 2 * a.S, a.thp, true);
      return;
    }
  }
  if constexpr (THV >= 0) return;  // launched only where the path above applies
  __syncthreads();
  for (int tile = run.t0; tile < run.t1; ++tile) {
    const int next = run.next(tile);
    xf(buf, S);
    pw_adj_combine(a, buf, tile);
    __syncthreads();
    pipe.issue(a.g, next, a.P);
    xf(buf, S);
    tile_store<T, XF::W, FAST, false>(a.g, tile, buf, a.P);
    __syncthreads();
    pipe.commit(a.g, next, a.P, buf);
    __syncthreads();
  }
}

// One transform along one axis, src -> dst (may alias), optional Neumann
// point weights before (divide) or after (multiply).
// PATH (FAST FP32 launches without point weights, chosen by the host): 1 =
// results straight to global memory (DCT-I / DST-I on one-species strided
// tiles), 2 = through the tile; only that path is compiled. 0: every path.
template <typename T, class XF, bool FAST, int PATH = 0>
__global__ __launch_bounds__(XF::THREADS, XF::MIN_WAVES_PER_EU) void k_single_m(SingleArgs<T> a, MfmaAxisDev ax) {
  to_member(a);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* buf = reinterpret_cast<T*>(smem_raw);
  XF xf(&a.g, &ax, reinterpret_cast<T*>(smem_raw + ax.fb_off));
  const Geom& g = a.g;
  const int ne = g.n * g.W;
  const int last = (int)(g.ntiles - 1);
  if constexpr (FAST && std::is_same<T, float>::value) {
    if (PATH != 0 || (!a.pre_divide_w && !a.post_multiply_w)) {
      // two tiles in flight: pipes A and B alternate
      TilePipe<T, XF::W, FAST, XF::XAX> pa, pb;
      const long long G = gridDim.x;
      auto nxt = [&](long long t) { return t < last ? t : last; };
      pa.issue(g, blockIdx.x, a.src);
      pb.issue(g, nxt(blockIdx.x + G), a.src);
      pa.commit(g, blockIdx.x, a.src, buf);
      __syncthreads();
      // results of DCT-I / DST-I transforms go straight to global memory
      // (x tiles hold their points along the rows: never straight to global memory)
      const bool direct =
          PATH == 1 || (PATH == 0 && !XF::XAX && ax.direct != 0 && g.spt == 1 && g.inner > 1);
      for (int tile = blockIdx.x; tile < g.ntiles; tile += 2 * G) {
        pa.issue(g, nxt(tile + 2 * G), a.src);
        if (direct) {
          xf.to_global(buf, a.dst + tile_ref(g, tile).base, g.inner);
        } else {
          xf(buf, g.spt);
          tile_store<T, XF::W, FAST, XF::XAX>(g, tile, buf, a.dst);
          __syncthreads();
        }
        pb.commit(g, nxt(tile + G), a.src, buf);
        __syncthreads();
        if (tile + G >= g.ntiles) break;
        pb.issue(g, nxt(tile + 3 * G), a.src);
        if (direct) {
          xf.to_global(buf, a.dst + tile_ref(g, tile + G).base, g.inner);
        } else {
          xf(buf, g.spt);
          tile_store<T, XF::W, FAST, XF::XAX>(g, tile + G, buf, a.dst);
          __syncthreads();
        }
        pa.commit(g, nxt(tile + 2 * G), a.src, buf);
        __syncthreads();
      }
      return;
    }
  }
  if constexpr (PATH != 0) return;
  TilePipe<T, XF::W, FAST, XF::XAX> pipe;
  pipe.issue(g, blockIdx.x, a.src);
  pipe.commit(g, blockIdx.x, a.src, buf);
  __syncthreads();
  for (int tile = blockIdx.x; tile < g.ntiles; tile += gridDim.x) {
    const int next = tile + gridDim.x < last ? tile + gridDim.x : last;
    pipe.issue(g, next, a.src);
    const TileRef tr = tile_ref(g, tile);
    if (a.pre_divide_w) {
      for (int e = threadIdx.x; e < ne; e += blockDim.x) {
        int j, w;
        unpack(g, e, j, w);
        long long idx;
        if (!elem(g, tr, j, w, idx)) continue;
        const T wt = T(point_weight(idx, a.n0, a.n1, a.n2));
        for (int s = 0; s < g.spt; ++s) buf[(s * g.n + j) * g.pitch + w] /= wt;
      }
      __syncthreads();
    }
    xf(buf, g.spt);
    if (a.post_multiply_w) {
      for (int e = threadIdx.x; e < ne; e += blockDim.x) {
        int j, w;
        unpack(g, e, j, w);
        long long idx;
        if (!elem(g, tr, j, w, idx)) continue;
        const T wt = T(point_weight(idx, a.n0, a.n1, a.n2));
        for (int s = 0; s < g.spt; ++s) buf[(s * g.n + j) * g.pitch + w] *= wt;
      }
      __syncthreads();
    }
    tile_store<T, XF::W, FAST, XF::XAX>(g, tile, buf, a.dst);
    __syncthreads();
    pipe.commit(g, next, a.src, buf);
    __syncthreads();
  }
}

}  // namespace sfrde
