// Device helpers shared by the gfx950 kernels: complex arithmetic and a batched
// in-LDS Stockham FFT (radix 8 / 4 / 2) for the channelizer and the beamspace DFT.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wbm {




__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by -j
__device__ __forceinline__ float2 cmul_mj(float2 a) { return make_float2(a.y, -a.x); }

__device__ __forceinline__ double2 dadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 dsub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 dmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ __forceinline__ double2 dcmulc(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 dscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }

// ---------------------------------------------------------------------------------------------
// Window placement (Eq. 18): u = M (d/lambda) sin(az) f_k/f_c, s = floor(u - (W-1)/2 + 1/2),
// evaluated in IEEE double with no contraction so that every kernel (and a host evaluation
// of the same expression) takes the same integer decision.
struct WindowGeom {
  int T, K, M, N, half_bin;
  double beta, dl;
  const double* sin_az;   // [T]
  const int* win;         // [T]
};

__device__ __forceinline__ void window_geom(double M, double dl, double sin_az, double beta,
                                            double ksh, double K, int W, double* u_out,
                                            int* s_out) {
#pragma clang fp contract(off)
  const double ratio = 1.0 + (beta * ksh) / K;
  const double u = ((M * dl) * sin_az) * ratio;
  const double c = u - 0.5 * (double)(W - 1);
  *s_out = (int)floor(c + 0.5);
  *u_out = u;
}

__device__ __forceinline__ void window_of(const WindowGeom& g, int t, int k, double* u, int* s) {
  const int ks = (k < g.K / 2) ? k : k - g.K;
  const double ksh = (double)ks + (g.half_bin ? 0.5 : 0.0);
  window_geom((double)g.M, g.dl, g.sin_az[t], g.beta, ksh, (double)g.K, g.win[t], u, s);
}

__device__ __forceinline__ int window_start(const WindowGeom& g, int t, int k) {
  double u;
  int s;
  window_of(g, t, k, &u, &s);
  return s;
}

// Windowed steering a~_i = M^-1/2 sum_{e<N} e^{j psi e}, psi = 2 pi (u - (s + i)) / M, by the
// Dirichlet closed form with sinpi / sincospi in FP64.
__device__ __forceinline__ double2 window_steering(const WindowGeom& g, double u, int s, int i) {
  const double xx = (u - (double)(s + i)) / (double)g.M;
  const double num = sinpi((double)g.N * xx), den = sinpi(xx);
  double mag = (den == 0.0) ? (double)g.N : num / den;
  mag /= sqrt((double)g.M);
  double sp, cp;
  sincospi((double)(g.N - 1) * xx, &sp, &cp);
  return make_double2(mag * cp, mag * sp);
}

// ---------------------------------------------------------------------------------------------
// Planar array (Sec. II-A, Sec. III-B): Nz x Nx elements, element (iz, ix) at vector index
// ix Nz + iz; an Mz x Mx beam grid, beam (mz, mx) at index mx Mz + mz; a Wz x Wx window, cell
// (iz_w, ix_w) at index ix_w Wz + iz_w.  Each axis places its window as the linear array
// does, from the direction cosines cx = cos(el) sin(az) and cz = sin(el).
struct UpaGeom {
  int T, K, Nz, Nx, Mz, Mx, half_bin;
  double beta, dl;
  const double* cx;   // [T]
  const double* cz;   // [T]
  const int* win;     // [T] Wz * Wx
  const int* wz;      // [T]
};

__device__ __forceinline__ void upa_window_of(const UpaGeom& g, int t, int k, double* uz,
                                              int* sz, double* ux, int* sx) {
  const int ks = (k < g.K / 2) ? k : k - g.K;
  const double ksh = (double)ks + (g.half_bin ? 0.5 : 0.0);
  const int Wz = g.wz[t], Wx = g.win[t] / Wz;
  window_geom((double)g.Mz, g.dl, g.cz[t], g.beta, ksh, (double)g.K, Wz, uz, sz);
  window_geom((double)g.Mx, g.dl, g.cx[t], g.beta, ksh, (double)g.K, Wx, ux, sx);
}

// One axis of the windowed steering: M^-1/2 sum_{e<N} e^{j psi e}, psi = 2 pi (u - m) / M
// (Dirichlet closed form; |u - m| < M for every window bin, so the only pole is u = m).
__device__ __forceinline__ double2 axis_steering(int N, int M, double u, int m) {
  const double xx = (u - (double)m) / (double)M;
  const double num = sinpi((double)N * xx), den = sinpi(xx);
  double mag = (den == 0.0) ? (double)N : num / den;
  mag /= sqrt((double)M);
  double sp, cp;
  sincospi((double)(N - 1) * xx, &sp, &cp);
  return make_double2(mag * cp, mag * sp);
}

// ---------------------------------------------------------------------------------------------
// Small DFTs in registers, forward sign: X[k] = sum_r v[r] exp(-2 pi i r k / R).  V is float2
// (the FP32 kernels) or double2 (the extended-precision kernels); the operations and their
// order are the same for both.

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double2 cmul_mj(double2 a) { return make_double2(a.y, -a.x); }

template <typename V>
struct Cplx;
template <>
struct Cplx<float2> {
  using S = float;
  __device__ __forceinline__ static float2 make(float a, float b) { return make_float2(a, b); }
};
template <>
struct Cplx<double2> {
  using S = double;
  __device__ __forceinline__ static double2 make(double a, double b) { return make_double2(a, b); }
};

// v * exp(-i pi m / 8), m in [0, 8) (a compile-time constant once loops are unrolled): the
// half-bin pre-twiddle h[tau] = exp(-i pi tau / n) at tau = j + r n / R factors into
// h[j] exp(-i pi r / R), so a channelizer thread keeps one table value per first-pass
// butterfly and applies these constant rotations to the rest of its inputs.
template <typename V>
__device__ __forceinline__ V rot_pi8(V v, int m) {
  constexpr double c[8] = {1.0, 0.92387953251128675613, 0.70710678118654752440,
                           0.38268343236508977173, 0.0, -0.38268343236508977173,
                           -0.70710678118654752440, -0.92387953251128675613};
  constexpr double s[8] = {0.0, 0.38268343236508977173, 0.70710678118654752440,
                           0.92387953251128675613, 1.0, 0.92387953251128675613,
                           0.70710678118654752440, 0.38268343236508977173};
  using S = typename Cplx<V>::S;
  if (m == 0) return v;
  if (m == 4) return cmul_mj(v);
  return cmul(v, Cplx<V>::make((S)c[m], (S)-s[m]));
}

template <typename V>
__device__ __forceinline__ void dft2(V* v) {
  V a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <typename V>
__device__ __forceinline__ void dft4(V& a0, V& a1, V& a2, V& a3) {
  V t0 = cadd(a0, a2), t1 = csub(a0, a2);
  V t2 = cadd(a1, a3), t3 = cmul_mj(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

template <typename V>
__device__ __forceinline__ void dft4(V* v) { dft4(v[0], v[1], v[2], v[3]); }

// odd outputs of the radix-8 split times exp(-2 pi i k / 8), k = 1, 2, 3
template <typename V>
__device__ __forceinline__ void rot8(V& o1, V& o2, V& o3) {
  using S = typename Cplx<V>::S;
  const S r = (S)0.70710678118654752440;
  o1 = Cplx<V>::make((o1.x + o1.y) * r, (o1.y - o1.x) * r);     // (1 - i)/sqrt2
  o2 = cmul_mj(o2);                                             // -i
  o3 = Cplx<V>::make((o3.y - o3.x) * r, -(o3.x + o3.y) * r);    // (-1 - i)/sqrt2
}

template <typename V>
__device__ __forceinline__ void dft8(V* v) {
  // even / odd split: E = DFT4(v0, v2, v4, v6), O = DFT4(v1, v3, v5, v7)
  V e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  V o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4(e0, e1, e2, e3);
  dft4(o0, o1, o2, o3);
  rot8(o1, o2, o3);
  v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
  v[1] = cadd(e1, o1); v[5] = csub(e1, o1);
  v[2] = cadd(e2, o2); v[6] = csub(e2, o2);
  v[3] = cadd(e3, o3); v[7] = csub(e3, o3);
}

template <int R, typename V>
__device__ __forceinline__ void dftR(V* v) {
  if constexpr (R == 2) dft2(v);
  else if constexpr (R == 4) dft4(v);
  else dft8(v);
}

// The same DFTs when the upper half of the inputs is zero (v[R/2 .. R-1] = 0, not read): the
// additions of those zeros are left out, which changes no value.
template <typename V>
__device__ __forceinline__ void dft4_zh(V& a0, V& a1, V& a2, V& a3) {
  const V x0 = a0, x1 = a1, t3 = cmul_mj(x1);
  a0 = cadd(x0, x1);
  a2 = csub(x0, x1);
  a1 = cadd(x0, t3);
  a3 = csub(x0, t3);
}

template <typename V>
__device__ __forceinline__ void dft8_zh(V* v) {
  V e0 = v[0], e1 = v[2], e2, e3;
  V o0 = v[1], o1 = v[3], o2, o3;
  dft4_zh(e0, e1, e2, e3);
  dft4_zh(o0, o1, o2, o3);
  rot8(o1, o2, o3);
  v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
  v[1] = cadd(e1, o1); v[5] = csub(e1, o1);
  v[2] = cadd(e2, o2); v[6] = csub(e2, o2);
  v[3] = cadd(e3, o3); v[7] = csub(e3, o3);
}

template <int R, typename V>
__device__ __forceinline__ void dftR_zh(V* v) {
  if constexpr (R == 2) {
    v[1] = v[0];
  } else if constexpr (R == 4) {
    dft4_zh(v[0], v[1], v[2], v[3]);
  } else {
    dft8_zh(v);
  }
}

// ---------------------------------------------------------------------------------------------
// Extended-precision storage of a complex FP64 value in 12 bytes: hi = its FP32 rounding
// (float2), lo = the remainder v - hi (exact in FP64) rounded to BF16, real part in the low
// half of a 32-bit word, imaginary part in the high half.  hi + lo carries the value to a
// relative error of at most about 2^-33 (lo <= 2^-25 |v|, BF16 keeps 8 significant bits),
// against 2^-25 for FP32 alone.
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

// hi = v rounded to FP32, lo = the two remainders rounded to BF16 (nearest, ties to even; the
// real part in the low half): one packed conversion instruction on gfx950
__device__ __forceinline__ void ext_split(double2 v, float2& hi, uint32_t& lo) {
  hi = make_float2((float)v.x, (float)v.y);
  const f32x2_t r = {(float)(v.x - (double)hi.x), (float)(v.y - (double)hi.y)};
  lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(r, bf16x2_t));
}

__device__ __forceinline__ double2 ext_join(float2 hi, uint32_t lo) {
  return make_double2((double)hi.x + (double)__uint_as_float(lo << 16),
                      (double)hi.y + (double)__uint_as_float(lo & 0xFFFF0000u));
}

// Batched forward DFT of `rows` rows of n = 2^LOGN points held across a workgroup of
// tile/8 threads, eight complex values per thread (Stockham autosort, radix 8 with one
// leading radix-2 or radix-4 pass).  Pass p of radix R over sub-length Ns: butterfly j of
// a row takes v[r] = x[j + r n/R], multiplies v[r] by exp(-2 pi i r (j mod Ns) / (Ns R)),
// applies the R-point DFT and stores v[r] at (j div Ns) Ns R + (j mod Ns) + r Ns.  Values
// live in registers inside a pass and in LDS between passes.  LDS position i of a row holds
// element i ^ ((i >> 3) & 31) (bits 0-4 XORed with bits 3-7: the stride-8 butterfly writes,
// the contiguous reads and the stride-64 blocks all land on distinct banks), and rows are PAD
// slots apart beyond n, chosen per shape for the kernel's output gather.
template <int LOGN, int LOGTILE, int PAD, typename V = float2>
struct Fft {
  static constexpr int n = 1 << LOGN;
  static constexpr int tile = 1 << LOGTILE;
  static constexpr int rows = tile / n;
  static constexpr int threads = tile / 8;
  static constexpr int rs = rows > 1 ? n + PAD : n;         // LDS row stride (complex)
  static constexpr int lds_complex = rows * rs;
  static constexpr int R0 = (LOGN % 3 == 1) ? 2 : ((LOGN % 3 == 2) ? 4 : 8);
  static constexpr int LOGR0 = (R0 == 2) ? 1 : (R0 == 4 ? 2 : 3);
  static_assert(LOGTILE >= LOGN && LOGTILE >= 3, "tile must hold a row and 8 values/thread");

  __device__ __forceinline__ static int addr(int row, int i) {
    return row * rs + (i ^ ((i >> 3) & 31));
  }

  // row and in-row butterfly index of this thread's p-th butterfly of a radix-R pass
  template <int LOGR>
  __device__ __forceinline__ static void bf(int p, int& row, int& j) {
    constexpr int LOGQ = LOGN - LOGR;
    const int b = threadIdx.x + p * threads;
    row = b >> LOGQ;
    j = b & ((1 << LOGQ) - 1);
  }

  // Radix-8 passes after the first, and the twiddles a thread applies in them: pass q
  // (stride 2^LOGNS, LOGNS = LOGR0 + 3 q) multiplies input r of its butterfly by
  // w^r, w = w_n^(kq * 2^(LOGN - LOGNS - 3)), kq = the butterfly's position within its stride.
  // They depend only on the thread, so a workgroup loads them once into registers: all seven
  // per pass up to two passes; from three passes on only w, w^2 and w^4 (table values), the
  // others formed by at most two complex products (w^3 = w^2 w, w^5 = w^4 w, w^6 = w^4 w^2,
  // w^7 = w^4 w^3) so that the large transforms stay within their register budget.
  static constexpr int NP = (LOGN - LOGR0) / 3;
  static constexpr int NPA = NP > 0 ? NP : 1;
  // FP64 values: always the three-twiddle form (register budget)
  static constexpr bool kCompact = NP >= 3 || sizeof(V) == sizeof(double2);
  static constexpr int NTW = kCompact ? 3 : 7;

  // tw[q * stride] = exp(-2 pi i q / n): an n-point table, or every stride-th entry of a
  // larger one.
  __device__ __forceinline__ static void load_twiddles(V (&tr)[NPA][NTW],
                                                       const V* __restrict__ tw,
                                                       int stride = 1) {
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      const int logns = LOGR0 + 3 * q;
      int row, j;
      bf<3>(0, row, j);
      const int step = (j & ((1 << logns) - 1)) << (LOGN - logns - 3);
      if constexpr (kCompact) {
        tr[q][0] = tw[step * stride];
        tr[q][1] = tw[2 * step * stride];
        tr[q][2] = tw[4 * step * stride];
      } else {
#pragma unroll
        for (int r = 1; r < 8; ++r) tr[q][r - 1] = tw[r * step * stride];
      }
    }
  }

  template <int R, int LOGR, int LOGNS, bool ZH = false>
  __device__ __forceinline__ static void compute_write(V (&v)[8], V* lds,
                                                       const V (&tr)[NPA][NTW]) {
#pragma unroll
    for (int p = 0; p < 8 / R; ++p) {
      int row, j;
      bf<LOGR>(p, row, j);
      V* b = v + p * R;
      const int k = j & ((1 << LOGNS) - 1);
      if constexpr (LOGNS > 0) {
        // only radix-8 passes follow the first (LOGNS == 0) pass: one butterfly per thread
        constexpr int q = (LOGNS - LOGR0) / 3;
        if constexpr (kCompact) {
          V w1 = tr[q][0], w2 = tr[q][1], w4 = tr[q][2];
          // empty register constraint: keeps the derived twiddles inside the tile loop (the
          // compiler would otherwise hoist them out and hold all seven per pass again)
          asm volatile("" : "+v"(w1.x), "+v"(w1.y), "+v"(w2.x), "+v"(w2.y), "+v"(w4.x), "+v"(w4.y));
          const V w3 = cmul(w2, w1);
          b[1] = cmul(b[1], w1);
          b[2] = cmul(b[2], w2);
          b[3] = cmul(b[3], w3);
          b[4] = cmul(b[4], w4);
          b[5] = cmul(b[5], cmul(w4, w1));
          b[6] = cmul(b[6], cmul(w4, w2));
          b[7] = cmul(b[7], cmul(w4, w3));
        } else {
#pragma unroll
          for (int r = 1; r < R; ++r) b[r] = cmul(b[r], tr[q][r - 1]);
        }
      }
      if constexpr (ZH && LOGNS == 0)
        dftR_zh<R>(b);
      else
        dftR<R>(b);
      const int base = ((j >> LOGNS) << (LOGNS + LOGR)) | k;
#pragma unroll
      for (int r = 0; r < R; ++r) lds[addr(row, base + (r << LOGNS))] = b[r];
    }
  }

  __device__ __forceinline__ static void read8(V (&v)[8], const V* lds) {
    constexpr int LOGQ = LOGN - 3;
    int row, j;
    bf<3>(0, row, j);
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = lds[addr(row, j + (r << LOGQ))];
  }

  template <int LOGNS>
  __device__ __forceinline__ static void rest(V (&v)[8], V* lds,
                                              const V (&tr)[NPA][NTW]) {
    if constexpr (LOGNS < LOGN) {
      __syncthreads();
      read8(v, lds);
      __syncthreads();
      compute_write<8, 3, LOGNS>(v, lds, tr);
      rest<LOGNS + 3>(v, lds, tr);
    }
  }

  // Index of the r-th input of this thread's p-th first-pass butterfly: (row, position).
  __device__ __forceinline__ static void first_input(int p, int r, int& row, int& pos) {
    int j;
    bf<LOGR0>(p, row, j);
    pos = j + (r << (LOGN - LOGR0));
  }

  // v holds the first-pass inputs (slot p*R0 + r <-> first_input(p, r)), tr the thread's
  // twiddles (load_twiddles); on return the transform of every row is in LDS in natural order
  // (addr(row, i)), visible to all threads.  ZH: the inputs at positions >= n/2 are zero (the
  // slots r >= R0/2 are not read).
  template <bool ZH = false>
  __device__ __forceinline__ static void run(V (&v)[8], V* lds,
                                             const V (&tr)[NPA][NTW]) {
    compute_write<R0, LOGR0, 0, ZH>(v, lds, tr);
    rest<LOGR0>(v, lds, tr);
    __syncthreads();
  }
};

}  // namespace wbm
