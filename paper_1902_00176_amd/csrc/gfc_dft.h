// gfc_dft.h - register-resident mixed-radix DFTs (radix 2, 3, 4, 5) for gfx950.
//
// A length-n DFT of a thread-private array is expanded at compile time. Lengths with two
// coprime factors n = A * B use the prime-factor (Good-Thomas) index maps, which need no
// twiddles between the factors (DftSel). Prime powers use decimation in time: n = R * Q, R
// sub-DFTs of length Q over the decimated inputs, a twiddle by w_n^(r k'), then Q DFTs of
// length R. Every index is a compile-time constant after
// unrolling, so the arrays live in VGPRs and every twiddle is an immediate. Twiddle
// constants are evaluated in float64 (constexpr series after exact octant reduction) and
// rounded once to float32. Multiplications by 1, -1, +-i and (+-1 +-i)/sqrt(2) are
// specialised away.
//
// SIGN = -1: forward transform X[k] = sum_n a[n] e^{-2 pi i n k / n};  SIGN = +1: inverse
// (unnormalised). Input and output are in natural order, in place.
#pragma once
#include <hip/hip_runtime.h>

namespace gfc {

struct cx {
  float x, y;
};

__host__ __device__ __forceinline__ cx cadd(cx a, cx b) { return {a.x + b.x, a.y + b.y}; }
__host__ __device__ __forceinline__ cx csub(cx a, cx b) { return {a.x - b.x, a.y - b.y}; }
__host__ __device__ __forceinline__ cx cmul(cx a, cx b) {
  return {__builtin_fmaf(a.x, b.x, -a.y * b.y), __builtin_fmaf(a.x, b.y, a.y * b.x)};
}
__host__ __device__ __forceinline__ cx cmulconj(cx a, cx b) {  // a * conj(b)
  return {__builtin_fmaf(a.x, b.x, a.y * b.y), __builtin_fmaf(a.y, b.x, -a.x * b.y)};
}
__host__ __device__ __forceinline__ cx cscale(cx a, float s) { return {a.x * s, a.y * s}; }
// multiply by SIGN * i
template <int SIGN>
__host__ __device__ __forceinline__ cx mul_si(cx a) {
  if constexpr (SIGN > 0) return {-a.y, a.x};
  else return {a.y, -a.x};
}

namespace detail {
constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double kH = 0.70710678118654752440084436210484903928;
constexpr double sin_series(double x) {
  double term = x, sum = x;
  for (int n = 1; n < 24; ++n) {
    term *= -x * x / double((2 * n) * (2 * n + 1));
    sum += term;
  }
  return sum;
}
constexpr double cos_series(double x) {
  double term = 1.0, sum = 1.0;
  for (int n = 1; n < 24; ++n) {
    term *= -x * x / double((2 * n - 1) * (2 * n));
    sum += term;
  }
  return sum;
}
// cos(2 pi e / n) (which = 0) or sin(2 pi e / n) (which = 1), reduced by octant exactly.
constexpr double cs2pi(long e, long n, int which) {
  e %= n;
  if (e < 0) e += n;
  const long e8 = 8 * e;
  const long q = e8 / n;                                   // octant 0..7
  const double r = kPi * double(e8 - q * n) / double(4 * n);  // in [0, pi/4)
  const double cr = cos_series(r), sr = sin_series(r);
  double c = 0.0, s = 0.0;
  switch (q) {
    case 0: c = cr; s = sr; break;
    case 1: c = kH * (cr - sr); s = kH * (cr + sr); break;
    case 2: c = -sr; s = cr; break;
    case 3: c = -kH * (cr + sr); s = kH * (cr - sr); break;
    case 4: c = -cr; s = -sr; break;
    case 5: c = kH * (sr - cr); s = -kH * (cr + sr); break;
    case 6: c = sr; s = -cr; break;
    default: c = kH * (cr + sr); s = kH * (sr - cr); break;
  }
  return which == 0 ? c : s;
}
}  // namespace detail

// v * w_N^E with w_N = e^{SIGN 2 pi i / N}
template <int N, int E, int SIGN>
__host__ __device__ __forceinline__ cx twc(cx v) {
  constexpr int e = ((E % N) + N) % N;
  if constexpr (e == 0) {
    return v;
  } else if constexpr (2 * e == N) {
    return {-v.x, -v.y};
  } else if constexpr (4 * e == N) {
    return mul_si<SIGN>(v);
  } else if constexpr (4 * e == 3 * N) {
    return mul_si<-SIGN>(v);
  } else if constexpr ((8 * e) % N == 0) {
    // odd multiple of pi/4: w = (c, s) with |c| = |s| = sqrt(1/2)
    constexpr double c = detail::cs2pi(e, N, 0);
    constexpr double s = SIGN * detail::cs2pi(e, N, 1);
    constexpr float h = float(detail::kH);
    if constexpr (c > 0 && s > 0) return {h * (v.x - v.y), h * (v.x + v.y)};
    else if constexpr (c > 0 && s < 0) return {h * (v.x + v.y), h * (v.y - v.x)};
    else if constexpr (c < 0 && s > 0) return {-h * (v.x + v.y), h * (v.x - v.y)};
    else return {h * (v.y - v.x), -h * (v.x + v.y)};
  } else {
    constexpr float c = float(detail::cs2pi(e, N, 0));
    constexpr float s = float(SIGN * detail::cs2pi(e, N, 1));
    return {__builtin_fmaf(v.x, c, -v.y * s), __builtin_fmaf(v.x, s, v.y * c)};
  }
}

constexpr int dft_radix(int n) {
  return (n % 4 == 0 && n > 4) ? 4 : (n % 2 == 0 && n > 2) ? 2 : (n % 3 == 0 && n > 3) ? 3
         : (n % 5 == 0 && n > 5) ? 5 : n;
}

// Coprime split n = A * B for the prime-factor (Good-Thomas) algorithm: A = the power of two
// in n, else the power of three; 1 when n is a prime power (then Cooley-Tukey is used).
constexpr int pow_part(int n, int p) {
  int a = 1;
  while (n % p == 0) {
    n /= p;
    a *= p;
  }
  return a;
}
constexpr int pfa_split(int n) {
  const int a2 = pow_part(n, 2);
  if (a2 > 1 && a2 < n) return a2;
  const int a3 = pow_part(n, 3);
  if (a3 > 1 && a3 < n) return a3;
  return 1;
}
// multiplicative inverse of a modulo m (a, m coprime), by search: compile time only
constexpr int inv_mod(int a, int m) {
  for (int x = 1; x < m; ++x)
    if ((a * x) % m == 1) return x;
  return 1;
}

template <int N, int SIGN>
struct Dft;

template <int SIGN>
struct Dft<1, SIGN> {
  __host__ __device__ __forceinline__ static void run(cx (&)[1]) {}
};

template <int SIGN>
struct Dft<2, SIGN> {
  __host__ __device__ __forceinline__ static void run(cx (&a)[2]) {
    const cx t = a[0];
    a[0] = cadd(t, a[1]);
    a[1] = csub(t, a[1]);
  }
};

template <int SIGN>
struct Dft<3, SIGN> {
  __host__ __device__ __forceinline__ static void run(cx (&a)[3]) {
    constexpr float s3 = 0.86602540378443864676f;
    const cx t1 = cadd(a[1], a[2]);
    const cx t2 = csub(a[1], a[2]);
    const cx m = {__builtin_fmaf(-0.5f, t1.x, a[0].x), __builtin_fmaf(-0.5f, t1.y, a[0].y)};
    const cx n = mul_si<SIGN>(cscale(t2, s3));
    a[0] = cadd(a[0], t1);
    a[1] = cadd(m, n);
    a[2] = csub(m, n);
  }
};

template <int SIGN>
struct Dft<4, SIGN> {
  __host__ __device__ __forceinline__ static void run(cx (&a)[4]) {
    const cx t0 = cadd(a[0], a[2]);
    const cx t1 = csub(a[0], a[2]);
    const cx t2 = cadd(a[1], a[3]);
    const cx t3 = mul_si<SIGN>(csub(a[1], a[3]));
    a[0] = cadd(t0, t2);
    a[2] = csub(t0, t2);
    a[1] = cadd(t1, t3);
    a[3] = csub(t1, t3);
  }
};

template <int SIGN>
struct Dft<5, SIGN> {
  __host__ __device__ __forceinline__ static void run(cx (&a)[5]) {
    constexpr float c1 = 0.30901699437494742410f;   // cos(2 pi / 5)
    constexpr float c2 = -0.80901699437494742410f;  // cos(4 pi / 5)
    constexpr float s1 = 0.95105651629515357212f;   // sin(2 pi / 5)
    constexpr float s2 = 0.58778525229247312917f;   // sin(4 pi / 5)
    const cx t1 = cadd(a[1], a[4]);
    const cx t2 = cadd(a[2], a[3]);
    const cx t3 = csub(a[1], a[4]);
    const cx t4 = csub(a[2], a[3]);
    const cx m1 = {__builtin_fmaf(c2, t2.x, __builtin_fmaf(c1, t1.x, a[0].x)),
                   __builtin_fmaf(c2, t2.y, __builtin_fmaf(c1, t1.y, a[0].y))};
    const cx m2 = {__builtin_fmaf(c1, t2.x, __builtin_fmaf(c2, t1.x, a[0].x)),
                   __builtin_fmaf(c1, t2.y, __builtin_fmaf(c2, t1.y, a[0].y))};
    const cx p1 = {__builtin_fmaf(s1, t3.x, s2 * t4.x), __builtin_fmaf(s1, t3.y, s2 * t4.y)};
    const cx p2 = {__builtin_fmaf(s2, t3.x, -s1 * t4.x), __builtin_fmaf(s2, t3.y, -s1 * t4.y)};
    const cx n1 = mul_si<SIGN>(p1);
    const cx n2 = mul_si<SIGN>(p2);
    a[0] = cadd(a[0], cadd(t1, t2));
    a[1] = cadd(m1, n1);
    a[4] = csub(m1, n1);
    a[2] = cadd(m2, n2);
    a[3] = csub(m2, n2);
  }
};

// Prime-factor algorithm for coprime N = A * B (no twiddles between the factors):
// input index n = (B n1 + A n2) mod N, output index k = (eA k1 + eB k2) mod N with
// eA = B (B^-1 mod A) (1 mod A, 0 mod B) and eB = A (A^-1 mod B) (0 mod A, 1 mod B); a
// length-A DFT over n1 for each n2, then a length-B DFT over n2 for each k1.
template <int N, int SIGN, int A = pfa_split(N)>
struct DftSel;

template <int N, int SIGN>
struct DftPfa {
  static constexpr int A = pfa_split(N);
  static constexpr int B = N / A;
  static constexpr int eA = (B * inv_mod(B % A, A)) % N;
  static constexpr int eB = (A * inv_mod(A % B, B)) % N;
  __host__ __device__ __forceinline__ static void run(cx (&a)[N]) {
    cx t[B][A];
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) {
#pragma unroll
      for (int n1 = 0; n1 < A; ++n1) t[n2][n1] = a[(B * n1 + A * n2) % N];
      DftSel<A, SIGN>::run(t[n2]);
    }
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
      cx c[B];
#pragma unroll
      for (int n2 = 0; n2 < B; ++n2) c[n2] = t[n2][k1];
      DftSel<B, SIGN>::run(c);
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) a[(eA * k1 + eB * k2) % N] = c[k2];
    }
  }
};

template <int N, int SIGN>
struct Dft {
  static constexpr int R = dft_radix(N);
  static constexpr int Q = N / R;
  static_assert(R * Q == N && R > 1 && Q > 1, "unsupported DFT length (must be 2^a 3^b 5^c)");

  template <int r, int K>
  __host__ __device__ __forceinline__ static void tw_row(cx (&t)[R], cx (&sub)[R][Q]) {
    if constexpr (r < R) {
      t[r] = twc<N, r * K, SIGN>(sub[r][K]);
      tw_row<r + 1, K>(t, sub);
    }
  }
  template <int K>
  __host__ __device__ __forceinline__ static void combine(cx (&a)[N], cx (&sub)[R][Q]) {
    if constexpr (K < Q) {
      cx t[R];
      tw_row<0, K>(t, sub);
      Dft<R, SIGN>::run(t);
#pragma unroll
      for (int s = 0; s < R; ++s) a[K + Q * s] = t[s];
      combine<K + 1>(a, sub);
    }
  }
  __host__ __device__ __forceinline__ static void run(cx (&a)[N]) {
    cx sub[R][Q];
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
      for (int m = 0; m < Q; ++m) sub[r][m] = a[R * m + r];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) Dft<Q, SIGN>::run(sub[r]);
    combine<0>(a, sub);
  }
};

// Dispatch: the prime-factor algorithm for lengths with a coprime split, Cooley-Tukey for
// prime powers (and the small radices themselves).
template <int N, int SIGN, int A>
struct DftSel {
  __host__ __device__ __forceinline__ static void run(cx (&a)[N]) {
    if constexpr (A > 1) DftPfa<N, SIGN>::run(a);
    else Dft<N, SIGN>::run(a);
  }
};

}  // namespace gfc
