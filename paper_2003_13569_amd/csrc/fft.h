// Hartley transforms of long periodic axes (N = 256, 512, 1024 points) as
// radix-8/4 complex FFTs in LDS.
//
// The periodic operator's eigenvalues satisfy lambda_k = lambda_{N-k}
// (Section 3.1), so the real Hartley basis cas(2 pi jk/N) = cos + sin
// diagonalises it like the complex Fourier basis of Alg. 1's fftn. Two real
// lines a, b of a tile are transformed together as one complex sequence
// z = a + i b: with Z = DFT(z) and Z'_k = Z_{(N-k) mod N},
//   H(a)_k = (Re Z_k + Re Z'_k - Im Z_k + Im Z'_k) / 2
//   H(b)_k = (Re Z_k - Re Z'_k + Im Z_k + Im Z'_k) / 2
// (Re and Im of the DFT of a real line are its cosine sum and minus its sine
// sum; the halves separate a and b by the conjugate symmetry of a real
// line's DFT). The Hartley transform is its own inverse up to 1/N, which the
// stage combine applies, so one routine serves both directions.
//
// The complex DFT is a Stockham autosort FFT (no bit reversal): stage by
// stage, butterfly j of span Ns reads x[j + r N/R], r < R, multiplies input r
// by e^{-2 pi i r k / (Ns R)} with k = j mod Ns, takes the radix-R DFT, and
// writes x[(j - k) R + k + r Ns]. One wavefront runs one pair of lines; its
// 64 lanes take butterflies lane, lane + 64, ... of every stage. Each stage
// reads all of its inputs before any output is written, so a single buffer of
// N complex values per wavefront suffices. Twiddles (cos, sin of 2 pi m / N)
// come from a table built in FP64 on the host.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.h"

namespace sfrde {

constexpr int FFT_MIN_N = 256;
constexpr int FFT_MAX_N = 1024;

// Radix-R DFT (e^{-2 pi i rk/R}) of v in place, R = 4 or 8.
template <typename T>
__device__ __forceinline__ void dft4(T& r0, T& i0, T& r1, T& i1, T& r2, T& i2, T& r3, T& i3) {
  const T t0r = r0 + r2, t0i = i0 + i2, t1r = r0 - r2, t1i = i0 - i2;
  const T t2r = r1 + r3, t2i = i1 + i3, t3r = r1 - r3, t3i = i1 - i3;
  r0 = t0r + t2r;
  i0 = t0i + t2i;
  r2 = t0r - t2r;
  i2 = t0i - t2i;
  // X1 = t1 - i t3, X3 = t1 + i t3
  r1 = t1r + t3i;
  i1 = t1i - t3r;
  r3 = t1r - t3i;
  i3 = t1i + t3r;
}

template <typename T, int R>
__device__ __forceinline__ void dft_r(T (&vr)[R], T (&vi)[R]) {
  if constexpr (R == 4) {
    dft4(vr[0], vi[0], vr[1], vi[1], vr[2], vi[2], vr[3], vi[3]);
  } else {
    static_assert(R == 8, "radix 4 or 8");
    // even and odd halves, then X_k = E_k + W8^k O_k, X_{k+4} = E_k - W8^k O_k
    T er[4] = {vr[0], vr[2], vr[4], vr[6]}, ei[4] = {vi[0], vi[2], vi[4], vi[6]};
    T orr[4] = {vr[1], vr[3], vr[5], vr[7]}, oi[4] = {vi[1], vi[3], vi[5], vi[7]};
    dft4(er[0], ei[0], er[1], ei[1], er[2], ei[2], er[3], ei[3]);
    dft4(orr[0], oi[0], orr[1], oi[1], orr[2], oi[2], orr[3], oi[3]);
    const T h = T(0.70710678118654752440);  // 1/sqrt(2)
    T wr[4], wi[4];
    wr[0] = orr[0];
    wi[0] = oi[0];
    wr[1] = (orr[1] + oi[1]) * h;  // (1 - i)/sqrt2
    wi[1] = (oi[1] - orr[1]) * h;
    wr[2] = oi[2];  // -i
    wi[2] = -orr[2];
    wr[3] = (oi[3] - orr[3]) * h;  // (-1 - i)/sqrt2
    wi[3] = -(orr[3] + oi[3]) * h;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      vr[k] = er[k] + wr[k];
      vi[k] = ei[k] + wi[k];
      vr[k + 4] = er[k] - wr[k];
      vi[k + 4] = ei[k] - wi[k];
    }
  }
}

// One Stockham stage of radix R and span NS on the wavefront's buffer
// (xr, xi) of N points. Block-wide barriers: every wavefront of the block
// runs the same stages; wavefronts without a line pair (`on` false) only
// take part in the barriers.
template <typename T, int N, int R, int NS>
__device__ __forceinline__ void fft_stage(T* xr, T* xi, const T* __restrict__ tw, int lane,
                                          bool on) {
  constexpr int NB = N / R;  // butterflies
  constexpr int B = NB / 64;  // per lane
  static_assert(B >= 1 && NB % 64 == 0, "at least one butterfly per lane");
  T vr[B][R], vi[B][R];
  if (on) {
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int j = lane + 64 * b;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        vr[b][r] = xr[j + r * NB];
        vi[b][r] = xi[j + r * NB];
      }
    }
  }
  __syncthreads();
  if (on) {
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int j = lane + 64 * b;
      const int k = j & (NS - 1);
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const int m = r * k * (N / (NS * R));  // < N
          const T c = tw[2 * m], s = tw[2 * m + 1];
          const T ar = vr[b][r], ai = vi[b][r];
          vr[b][r] = ar * c + ai * s;  // times e^{-i theta}
          vi[b][r] = ai * c - ar * s;
        }
      }
      dft_r<T, R>(vr[b], vi[b]);
      const int base = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        xr[base + r * NS] = vr[b][r];
        xi[base + r * NS] = vi[b][r];
      }
    }
  }
  __syncthreads();
}

// Complex DFT of the wavefront's buffer, natural order in and out.
template <typename T, int N>
__device__ __forceinline__ void fft_wave(T* xr, T* xi, const T* __restrict__ tw, int lane,
                                         bool on) {
  if constexpr (N == 256) {
    fft_stage<T, N, 4, 1>(xr, xi, tw, lane, on);
    fft_stage<T, N, 4, 4>(xr, xi, tw, lane, on);
    fft_stage<T, N, 4, 16>(xr, xi, tw, lane, on);
    fft_stage<T, N, 4, 64>(xr, xi, tw, lane, on);
  } else if constexpr (N == 512) {
    fft_stage<T, N, 8, 1>(xr, xi, tw, lane, on);
    fft_stage<T, N, 8, 8>(xr, xi, tw, lane, on);
    fft_stage<T, N, 8, 64>(xr, xi, tw, lane, on);
  } else {
    static_assert(N == 1024, "N = 256, 512 or 1024");
    fft_stage<T, N, 8, 1>(xr, xi, tw, lane, on);
    fft_stage<T, N, 8, 8>(xr, xi, tw, lane, on);
    fft_stage<T, N, 4, 64>(xr, xi, tw, lane, on);
    fft_stage<T, N, 4, 256>(xr, xi, tw, lane, on);
  }
}

// Lines per tile of an FFT axis and the LDS the kernels need: tiles hold W
// lines of spt species (x axis: spt = S, W = 2 for S <= 2 else 1; strided
// axes: spt = 1, W = 4), one wavefront per pair of the tile's spt * W lines;
// the block has FFT_THREADS threads (at least one wavefront per pair), all of
// which take part in the tile's loads, stores and pointwise stages.
constexpr int FFT_THREADS = 256;
__host__ __device__ constexpr int fft_pairs(int spt, int W) { return (spt * W + 1) / 2; }
template <typename T>
constexpr size_t fft_lds_bytes(int spt, int n, int W, int pitch) {
  return ((size_t)spt * n * pitch + (size_t)fft_pairs(spt, W) * 2 * n) * sizeof(T);
}

// The transform functor of the tile kernels (kernels.h): Hartley transform of
// every line of the tile buf[s][j][w], in place. Wavefront q < pairs runs the
// pair of lines 2q, 2q + 1; the pair buffers follow the tile in LDS.
template <typename T>
struct FftXf {
  const Geom* g;
  const T* tw;  // [N][2] cos, sin of 2 pi m / N
  __device__ __forceinline__ void operator()(T* buf, int S) {
    const int n = g->n, W = g->W, pitch = g->pitch;
    const int L = S * W;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const bool on = wave < fft_pairs(S, W);
    const int l0 = 2 * wave, l1 = 2 * wave + 1;
    const bool has1 = l1 < L;
    T* xr = buf + (size_t)S * n * pitch + (size_t)(on ? wave : 0) * 2 * n;
    T* xi = xr + n;
    T* a = buf + (size_t)(l0 / W) * n * pitch + (l0 % W);
    T* b = buf + (size_t)(l1 / W) * n * pitch + (l1 % W);
    if (on) {
      for (int j = lane; j < n; j += 64) {
        xr[j] = a[j * pitch];
        xi[j] = has1 ? b[j * pitch] : T(0);
      }
    }
    __syncthreads();
    switch (n) {
      case 256: fft_wave<T, 256>(xr, xi, tw, lane, on); break;
      case 512: fft_wave<T, 512>(xr, xi, tw, lane, on); break;
      default: fft_wave<T, 1024>(xr, xi, tw, lane, on); break;
    }
    if (on) {
      for (int k = lane; k < n; k += 64) {
        const int kk = (n - k) & (n - 1);
        const T zr = xr[k], zi = xi[k], wr = xr[kk], wi = xi[kk];
        a[k * pitch] = T(0.5) * ((zr + wr) - (zi - wi));
        if (has1) b[k * pitch] = T(0.5) * ((zr - wr) + (zi + wi));
      }
    }
    __syncthreads();
  }
};

}  // namespace sfrde
