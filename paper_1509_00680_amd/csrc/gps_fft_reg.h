// In-register FFT codelets with compile-time length (used by the two-level
// FFT passes).  Roots of unity are compile-time constants evaluated by the
// C++ front end in binary64 (Taylor series on the first octant), so the
// unrolled butterflies carry literal twiddles.
#pragma once

#include "gps_device.h"

namespace gps {

// ---- constexpr cos/sin(2 pi m / n) ------------------------------------------
__host__ __device__ constexpr double ce_sin_series(double x) {
  double term = x, sum = x;
  for (int i = 1; i < 14; ++i) {
    term *= -x * x / ((2.0 * i) * (2.0 * i + 1.0));
    sum += term;
  }
  return sum;
}
__host__ __device__ constexpr double ce_cos_series(double x) {
  double term = 1.0, sum = 1.0;
  for (int i = 1; i < 14; ++i) {
    term *= -x * x / ((2.0 * i - 1.0) * (2.0 * i));
    sum += term;
  }
  return sum;
}
// angle 2 pi m/n reduced to the first octant by exact integer symmetries
__host__ __device__ constexpr void ce_root(long long m, long long n, double* c, double* s) {
  m %= n;
  if (m < 0) m += n;
  // quadrant: multiply by 4 to compare with n exactly
  long long q = (4 * m) / n;            // 0..3
  long long r4 = 4 * m - q * n;         // angle within the quadrant, in units of 2 pi/(4n)
  // theta = 2 pi m/n = q pi/2 + phi, phi = (pi/2) r4/n
  bool swap = 2 * r4 > n;               // phi > pi/4: use pi/2 - phi
  long long num = swap ? (n - r4) : r4;
  double phi = 1.5707963267948966192313216916398 * (double)num / (double)n;
  double sp = ce_sin_series(phi), cp = ce_cos_series(phi);
  if (swap) { double t = sp; sp = cp; cp = t; }
  double cc = cp, ss = sp;
  if (q == 1) { cc = -sp; ss = cp; }
  else if (q == 2) { cc = -cp; ss = -sp; }
  else if (q == 3) { cc = sp; ss = -cp; }
  *c = cc;
  *s = ss;
}

// w_N^e = exp(-2 pi i e/N) (forward) or its conjugate (inverse).  Called with
// indices that are constant after unrolling, so the series folds to literals.
template <typename T, int N, bool INV>
__device__ __forceinline__ cplx<T> croot(int e) {
  double c = 0.0, s = 0.0;
  ce_root(e, N, &c, &s);
  return cmk(T(c), T(INV ? s : -s));
}

// v * w_N^e for an exponent that is constant after unrolling: the quarter
// turns (1, -1, -i, +i) become swaps and sign changes instead of a full
// complex multiplication (whose products with 0 the compiler must keep).
template <typename T, int N, bool INV>
__device__ __forceinline__ cplx<T> twiddle(cplx<T> v, int e) {
  e %= N;
  if (e == 0) return v;
  if (2 * e == N) return cmk(-v.x, -v.y);
  const bool minus_i = (4 * e == N) != INV;         // w = -i (else +i) when a quarter turn
  if (4 * e == N || 4 * e == 3 * N) return minus_i ? cmk(v.y, -v.x) : cmk(-v.y, v.x);
  return cmul(v, croot<T, N, INV>(e));
}

// ---- small DFTs (radix butterflies) ---------------------------------------
template <int R> struct OddRoots;
template <> struct OddRoots<3> {
  static constexpr double c[2] = {1.0, -0.5};
  static constexpr double s[2] = {0.0, 0.86602540378443864676};
};
template <> struct OddRoots<5> {
  static constexpr double c[3] = {1.0, 0.30901699437494742410, -0.80901699437494742410};
  static constexpr double s[3] = {0.0, 0.95105651629515357212, 0.58778525229247312917};
};

template <typename T, bool INV, int R>
__device__ __forceinline__ void rdft(cplx<T>* x) {
  if constexpr (R == 2) {
    const cplx<T> a = x[0];
    x[0] = cadd(a, x[1]);
    x[1] = csub(a, x[1]);
  } else if constexpr (R == 4) {
    const cplx<T> a0 = cadd(x[0], x[2]), a1 = csub(x[0], x[2]);
    const cplx<T> a2 = cadd(x[1], x[3]), a3 = csub(x[1], x[3]);
    const cplx<T> ja3 = INV ? cmk(-a3.y, a3.x) : cmk(a3.y, -a3.x);
    x[0] = cadd(a0, a2);
    x[2] = csub(a0, a2);
    x[1] = cadd(a1, ja3);
    x[3] = csub(a1, ja3);
  } else {
    static_assert(R == 3 || R == 5, "radix");
    constexpr int H = (R - 1) / 2;
    cplx<T> a[H + 1], b[H + 1];
#pragma unroll
    for (int n = 1; n <= H; ++n) {
      a[n] = cadd(x[n], x[R - n]);
      b[n] = csub(x[n], x[R - n]);
    }
    const cplx<T> x0 = x[0];
    cplx<T> y0 = x0;
#pragma unroll
    for (int n = 1; n <= H; ++n) y0 = cadd(y0, a[n]);
#pragma unroll
    for (int k = 1; k <= H; ++k) {
      cplx<T> re = x0, im = cmk(T(0), T(0));
#pragma unroll
      for (int n = 1; n <= H; ++n) {
        const int m = (n * k) % R;
        const int mf = m <= H ? m : R - m;
        re = cadd(re, cscale(a[n], T(OddRoots<R>::c[mf])));
        im = cadd(im, cscale(b[n], T(m <= H ? OddRoots<R>::s[mf] : -OddRoots<R>::s[mf])));
      }
      const cplx<T> mi = cmk(im.y, -im.x);   // -i * im
      if (INV) {
        x[k] = csub(re, mi);
        x[R - k] = cadd(re, mi);
      } else {
        x[k] = cadd(re, mi);
        x[R - k] = csub(re, mi);
      }
    }
    x[0] = y0;
  }
}

// ---- register Stockham over a compile-time radix list -----------------------
template <typename T, bool INV, int N, int Ns, int... Rs> struct RegFFT {
  static __device__ __forceinline__ void run(cplx<T>*) {}
};
template <typename T, bool INV, int N, int Ns, int R, int... Rest>
struct RegFFT<T, INV, N, Ns, R, Rest...> {
  static __device__ __forceinline__ void run(cplx<T>* x) {
    cplx<T> y[N];
#pragma unroll
    for (int j = 0; j < N / R; ++j) {
      const int k = j % Ns;
      cplx<T> v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        v[r] = x[j + r * (N / R)];
        if (r > 0 && k > 0) v[r] = twiddle<T, Ns * R, INV>(v[r], r * k);
      }
      rdft<T, INV, R>(v);
      const int base = (j / Ns) * Ns * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) y[base + r * Ns] = v[r];
    }
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = y[i];
    RegFFT<T, INV, N, Ns * R, Rest...>::run(x);
  }
};

// ---- prime-factor (Good-Thomas) codelet for N = N1 N2 with gcd(N1, N2) = 1 --
// Input n = (N2 n1 + N1 n2) mod N is read as a N1 x N2 array; N1-point DFTs
// along n1, then N2-point DFTs along n2, and output (k1, k2) is X[k] with
// k = k1 mod N1 = k2 mod N2 (Chinese remainder theorem).  The exponent of
// w_N factors exactly into w_N1^(n1 k1) w_N2^(n2 k2), so no twiddle factor
// sits between the two stages.  All indices are compile-time after unrolling.
// Inverse of a modulo m (gcd(a, m) = 1), evaluated in constant expressions.
__host__ __device__ constexpr int ce_modinv(int a, int m) {
  int r = 1;
  while ((a * r) % m != 1 % m) ++r;
  return r;
}
// CRT idempotents: E1 = 1 mod N1, 0 mod N2; E2 = 0 mod N1, 1 mod N2.  The
// output index of (k1, k2) is (k1 E1 + k2 E2) mod N, plain arithmetic on
// unrolled constants.
template <int N1, int N2> struct PfaMap {
  static constexpr int E1 = N2 * ce_modinv(N2 % N1, N1);
  static constexpr int E2 = N1 * ce_modinv(N1 % N2, N2);
};

template <typename T, bool INV, int N> struct Codelet;

template <typename T, bool INV, int N1, int N2> struct PfaFFT {
  static __device__ __forceinline__ void run(cplx<T>* x) {
    constexpr int N = N1 * N2;
    cplx<T> y[N];
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) {
      cplx<T> v[N1];
#pragma unroll
      for (int n1 = 0; n1 < N1; ++n1) v[n1] = x[(N2 * n1 + N1 * n2) % N];
      Codelet<T, INV, N1>::run(v);
#pragma unroll
      for (int k1 = 0; k1 < N1; ++k1) y[k1 * N2 + n2] = v[k1];
    }
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) {
      cplx<T> v[N2];
#pragma unroll
      for (int n2 = 0; n2 < N2; ++n2) v[n2] = y[k1 * N2 + n2];
      Codelet<T, INV, N2>::run(v);
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2)
        x[(k1 * PfaMap<N1, N2>::E1 + k2 * PfaMap<N1, N2>::E2) % N] = v[k2];
    }
  }
};

// Radix lists of the codelet lengths (prime-factor form where N splits into
// coprime factors).
#define GPS_CODELET(N, ...)                                                         \
  template <typename T, bool INV> struct Codelet<T, INV, N> {                       \
    static __device__ __forceinline__ void run(cplx<T>* x) {                        \
      RegFFT<T, INV, N, 1, __VA_ARGS__>::run(x);                                    \
    }                                                                               \
  };
#define GPS_PFA_CODELET(N, N1, N2)                                                  \
  template <typename T, bool INV> struct Codelet<T, INV, N> {                       \
    static __device__ __forceinline__ void run(cplx<T>* x) {                        \
      PfaFFT<T, INV, N1, N2>::run(x);                                               \
    }                                                                               \
  };
GPS_CODELET(2, 2)
GPS_CODELET(3, 3)
GPS_CODELET(4, 4)
GPS_CODELET(5, 5)
GPS_CODELET(8, 4, 2)
GPS_CODELET(16, 4, 4)
GPS_CODELET(32, 4, 4, 2)
GPS_PFA_CODELET(6, 2, 3)
GPS_PFA_CODELET(10, 2, 5)
GPS_PFA_CODELET(12, 4, 3)
GPS_PFA_CODELET(20, 4, 5)
GPS_PFA_CODELET(24, 8, 3)
#undef GPS_CODELET
#undef GPS_PFA_CODELET

// Natural-order DFT of N values held in registers.
template <typename T, bool INV, int N>
__device__ __forceinline__ void reg_fft(cplx<T>* x) {
  Codelet<T, INV, N>::run(x);
}

}  // namespace gps
