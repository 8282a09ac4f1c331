// pwfs_dft.h -- in-register mixed-radix DFTs and quad-lane helpers for gfx950.
//
// Every transform here is fully unrolled at compile time: the data live in
// registers of one lane, all twiddles are compile-time FP64 values rounded
// to FP32, trivial twiddles (1, -1, +-i) are never multiplied, and lengths
// with coprime factors use the twiddle-free prime-factor split.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <utility>

namespace pwfs {

struct alignas(8) cpx {
  float re, im;
};

__device__ __forceinline__ cpx cadd(cpx a, cpx b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cpx csub(cpx a, cpx b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cpx cmul(cpx a, cpx b) {
  return {fmaf(a.re, b.re, -a.im * b.im), fmaf(a.re, b.im, a.im * b.re)};
}
// a * b + c (four FMAs)
__device__ __forceinline__ cpx cfma(cpx a, cpx b, cpx c) {
  return {fmaf(a.re, b.re, fmaf(-a.im, b.im, c.re)), fmaf(a.re, b.im, fmaf(a.im, b.re, c.im))};
}
// a * conj(b)
__device__ __forceinline__ cpx cmulc(cpx a, cpx b) {
  return {fmaf(a.re, b.re, a.im * b.im), fmaf(a.im, b.re, -a.re * b.im)};
}

// ---------------------------------------------------------------------------
// Compile-time sin / cos of the rational angle 2 pi n / d in double precision.
// The angle is reduced exactly with integers to |r| <= pi / 4 before a Taylor
// series, so every constant is correctly rounded to well below FP32 ulp.
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double taylor_sin(double x) {
  double x2 = x * x, term = x, sum = x;
  for (int k = 1; k < 14; ++k) {
    term *= -x2 / double((2 * k) * (2 * k + 1));
    sum += term;
  }
  return sum;
}
constexpr double taylor_cos(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int k = 1; k < 14; ++k) {
    term *= -x2 / double((2 * k - 1) * (2 * k));
    sum += term;
  }
  return sum;
}
// cos and sin of 2 pi n / d.
constexpr double cos_frac(long n, long d) {
  n %= d;
  if (n < 0) n += d;
  long q = (8 * n + d) / (2 * d);  // nearest quarter turn
  double r = 2.0 * kPi * double(4 * n - q * d) / double(4 * d);
  double c = taylor_cos(r), s = taylor_sin(r);
  switch (q & 3) {
    case 0: return c;
    case 1: return -s;
    case 2: return -c;
    default: return s;
  }
}
constexpr double sin_frac(long n, long d) {
  n %= d;
  if (n < 0) n += d;
  long q = (8 * n + d) / (2 * d);
  double r = 2.0 * kPi * double(4 * n - q * d) / double(4 * d);
  double c = taylor_cos(r), s = taylor_sin(r);
  switch (q & 3) {
    case 0: return s;
    case 1: return c;
    case 2: return -s;
    default: return -c;
  }
}

// ---------------------------------------------------------------------------
// Unrolling helper: f(std::integral_constant<int, I>{}) for I in [0, N).
template <int Base, typename F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, Base + I>{}), ...);
}
template <int Begin, int End, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl<Begin>(f, std::make_integer_sequence<int, End - Begin>{});
}

// v * w with w = exp(-2 pi i DIR n / d): trivial angles are exact.
template <long n, long d, int DIR>
__device__ __forceinline__ cpx twiddle(cpx v) {
  constexpr long nn = ((n % d) + d) % d;
  if constexpr (nn == 0) {
    return v;
  } else if constexpr (4 * nn == d) {         // -i DIR
    return DIR > 0 ? cpx{v.im, -v.re} : cpx{-v.im, v.re};
  } else if constexpr (2 * nn == d) {
    return cpx{-v.re, -v.im};
  } else if constexpr (4 * nn == 3 * d) {     // +i DIR
    return DIR > 0 ? cpx{-v.im, v.re} : cpx{v.im, -v.re};
  } else {
    constexpr float c = float(cos_frac(nn, d));
    constexpr float s = float(-DIR * sin_frac(nn, d));
    return {fmaf(v.re, c, -v.im * s), fmaf(v.re, s, v.im * c)};
  }
}

// Small radices -------------------------------------------------------------
// All compute X[k] = sum_m x[m] exp(-2 pi i DIR m k / R), natural order.
template <int R, int DIR>
struct Radix;

template <int DIR>
struct Radix<1, DIR> {
  __device__ __forceinline__ static void run(cpx*) {}
};

template <int DIR>
struct Radix<2, DIR> {
  __device__ __forceinline__ static void run(cpx* x) {
    cpx a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  }
};

template <int DIR>
struct Radix<3, DIR> {
  __device__ __forceinline__ static void run(cpx* x) {
    constexpr float s3 = float(0.86602540378443864676372317075294);  // sin(2 pi / 3)
    cpx s = cadd(x[1], x[2]), d = csub(x[1], x[2]);
    cpx a = {x[0].re - 0.5f * s.re, x[0].im - 0.5f * s.im};
    cpx b = {s3 * d.re, s3 * d.im};
    x[0] = cadd(x[0], s);
    // X1 = a - i DIR b, X2 = a + i DIR b
    x[1] = DIR > 0 ? cpx{a.re + b.im, a.im - b.re} : cpx{a.re - b.im, a.im + b.re};
    x[2] = DIR > 0 ? cpx{a.re - b.im, a.im + b.re} : cpx{a.re + b.im, a.im - b.re};
  }
};

template <int DIR>
struct Radix<4, DIR> {
  __device__ __forceinline__ static void run(cpx* x) {
    cpx t0 = cadd(x[0], x[2]), t1 = cadd(x[1], x[3]);
    cpx t2 = csub(x[0], x[2]), t3 = csub(x[1], x[3]);
    // t3 * (-i DIR)
    cpx t3r = DIR > 0 ? cpx{t3.im, -t3.re} : cpx{-t3.im, t3.re};
    x[0] = cadd(t0, t1);
    x[2] = csub(t0, t1);
    x[1] = cadd(t2, t3r);
    x[3] = csub(t2, t3r);
  }
};

template <int DIR>
struct Radix<5, DIR> {
  __device__ __forceinline__ static void run(cpx* x) {
    constexpr float c1 = float(0.30901699437494742410229341718282);   // cos(2 pi / 5)
    constexpr float c2 = float(-0.80901699437494742410229341718282);  // cos(4 pi / 5)
    constexpr float s1 = float(0.95105651629515357211643933337938);   // sin(2 pi / 5)
    constexpr float s2 = float(0.58778525229247312916870595463907);   // sin(4 pi / 5)
    cpx sA = cadd(x[1], x[4]), dA = csub(x[1], x[4]);
    cpx sB = cadd(x[2], x[3]), dB = csub(x[2], x[3]);
    cpx x0 = x[0];
    cpx a1 = {fmaf(c2, sB.re, fmaf(c1, sA.re, x0.re)), fmaf(c2, sB.im, fmaf(c1, sA.im, x0.im))};
    cpx a2 = {fmaf(c1, sB.re, fmaf(c2, sA.re, x0.re)), fmaf(c1, sB.im, fmaf(c2, sA.im, x0.im))};
    cpx b1 = {fmaf(s2, dB.re, s1 * dA.re), fmaf(s2, dB.im, s1 * dA.im)};
    cpx b2 = {fmaf(-s1, dB.re, s2 * dA.re), fmaf(-s1, dB.im, s2 * dA.im)};
    x[0] = {x0.re + sA.re + sB.re, x0.im + sA.im + sB.im};
    // X_k = a_k - i DIR b_k, X_{5-k} = a_k + i DIR b_k
    if constexpr (DIR > 0) {
      x[1] = {a1.re + b1.im, a1.im - b1.re};
      x[4] = {a1.re - b1.im, a1.im + b1.re};
      x[2] = {a2.re + b2.im, a2.im - b2.re};
      x[3] = {a2.re - b2.im, a2.im + b2.re};
    } else {
      x[1] = {a1.re - b1.im, a1.im + b1.re};
      x[4] = {a1.re + b1.im, a1.im - b1.re};
      x[2] = {a2.re - b2.im, a2.im + b2.re};
      x[3] = {a2.re + b2.im, a2.im - b2.re};
    }
  }
};

constexpr int first_radix(int n) {
  if (n % 4 == 0 && n != 8) return 4;
  if (n % 2 == 0) return 2;
  if (n % 3 == 0) return 3;
  if (n % 5 == 0) return 5;
  return n;
}

// Largest power of the smallest prime factor of n, or 0 when n is itself a
// prime power (no split into coprime factors).
constexpr int coprime_part(int n) {
  for (int p = 2; p <= n; ++p) {
    if (n % p == 0) {
      int q = p;
      while (n % (q * p) == 0) q *= p;
      return q == n ? 0 : q;
    }
  }
  return 0;
}
// a^{-1} mod m for gcd(a, m) = 1, m > 1.
constexpr int inverse_mod(int a, int m) {
  for (int x = 1; x < m; ++x)
    if ((a * x) % m == 1) return x;
  return 0;
}

// Composite length E.  With coprime factors E = N1 N2 the prime-factor
// (Good-Thomas) split needs no twiddles: input n = (N2 n1 + N1 n2) mod E,
// output k = (N2 u k1 + N1 v k2) mod E with u = N2^{-1} mod N1 and
// v = N1^{-1} mod N2, since then w_E^{nk} = w_N1^{n1 k1} w_N2^{n2 k2}.
// Prime powers use decimation in time, E = R * Q:
//   X[k1 + Q k2] = sum_r w_E^{r k1} w_R^{r k2} DFT_Q(x[R q + r])[k1]
template <int E, int DIR>
struct Dft {
  static constexpr int N1 = coprime_part(E);
  static constexpr int R = first_radix(E);
  static constexpr int Q = E / R;
  __device__ __forceinline__ static void run(cpx (&x)[E]) {
    if constexpr (N1 > 0) {
      constexpr int N2 = E / N1;
      constexpr int U = inverse_mod(N2 % N1, N1);
      constexpr int V = inverse_mod(N1 % N2, N2);
      static_assert((N2 * U) % N1 == 1 && (N1 * V) % N2 == 1, "factors not coprime");
      cpx t[N1][N2];
      static_for<0, N1>([&](auto n1_) {
        constexpr int n1 = decltype(n1_)::value;
        static_for<0, N2>([&](auto n2_) {
          constexpr int n2 = decltype(n2_)::value;
          t[n1][n2] = x[(N2 * n1 + N1 * n2) % E];
        });
        Dft<N2, DIR>::run(t[n1]);
      });
      static_for<0, N2>([&](auto k2_) {
        constexpr int k2 = decltype(k2_)::value;
        cpx u[N1];
        static_for<0, N1>([&](auto n1_) {
          constexpr int n1 = decltype(n1_)::value;
          u[n1] = t[n1][k2];
        });
        Dft<N1, DIR>::run(u);
        static_for<0, N1>([&](auto k1_) {
          constexpr int k1 = decltype(k1_)::value;
          x[(N2 * U * k1 + N1 * V * k2) % E] = u[k1];
        });
      });
    } else if constexpr (Q == 1) {
      Radix<R, DIR>::run(x);
    } else {
      cpx t[R][Q];
      static_for<0, R>([&](auto r_) {
        constexpr int r = decltype(r_)::value;
        static_for<0, Q>([&](auto q_) {
          constexpr int q = decltype(q_)::value;
          t[r][q] = x[R * q + r];
        });
        Dft<Q, DIR>::run(t[r]);
        static_for<0, Q>([&](auto k_) {
          constexpr int k1 = decltype(k_)::value;
          t[r][k1] = twiddle<long(r) * k1, E, DIR>(t[r][k1]);
        });
      });
      static_for<0, Q>([&](auto k_) {
        constexpr int k1 = decltype(k_)::value;
        cpx u[R];
        static_for<0, R>([&](auto r_) {
          constexpr int r = decltype(r_)::value;
          u[r] = t[r][k1];
        });
        Radix<R, DIR>::run(u);
        static_for<0, R>([&](auto k2_) {
          constexpr int k2 = decltype(k2_)::value;
          x[k1 + Q * k2] = u[k2];
        });
      });
    }
  }
};

template <int DIR>
struct Dft<1, DIR> {
  __device__ __forceinline__ static void run(cpx (&)[1]) {}
};

// ---------------------------------------------------------------------------
// Cross-lane moves.  DPP quad_perm: lane i of each quad reads lane perm[i].
template <int CTRL>
__device__ __forceinline__ float quad_perm(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}
// Lane i reads lane i ^ 4 (partner quad of an 8-lane team), ds_swizzle bit mode.
__device__ __forceinline__ float swap_quads(float v) {
  return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x101F));
}

// Lane i reads lane i ^ 16 (partner projection of a 32-lane team), ds_swizzle bit mode.
__device__ __forceinline__ float swap_halves(float v) {
  return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F));
}

// Three-tap lane mix V = v + a v' + b v'', with v' and v'' the values of v on
// the lanes that the DPP controls PL and MI select (quad form: lanes l + 1 and
// l - 1 mod 4), for two values v0, v1 of the same lanes in one block.  Each
// neighbour value is read through the DPP operand of the multiply-add itself
// instead of a separate DPP move (ten VALU instructions per mix instead of
// twelve).  The leading s_nop 1 gives the two wait states a DPP read needs
// after a VALU write of its source, once for both mixes; inside the block no
// DPP source is written, and every lane is active wherever this is used.
#define PWFS_MIX3x2_ASM(PL, MI)                                                \
  "s_nop 1\n\t"                                                                \
  "v_mul_f32_dpp %0, %4, %6 " PL " row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"   \
  "v_mul_f32_dpp %1, %5, %6 " PL " row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"   \
  "v_mul_f32_dpp %2, %10, %12 " PL " row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"   \
  "v_mul_f32_dpp %3, %11, %12 " PL " row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"   \
  "v_fmac_f32_dpp %0, -%5, %7 " PL " row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t" \
  "v_fmac_f32_dpp %1, %4, %7 " PL " row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"  \
  "v_fmac_f32_dpp %2, -%11, %13 " PL " row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t" \
  "v_fmac_f32_dpp %3, %10, %13 " PL " row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"  \
  "v_fmac_f32_dpp %0, %4, %8 " MI " row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"  \
  "v_fmac_f32_dpp %1, %5, %8 " MI " row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"  \
  "v_fmac_f32_dpp %2, %10, %14 " MI " row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"  \
  "v_fmac_f32_dpp %3, %11, %14 " MI " row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"  \
  "v_fmac_f32_dpp %0, -%5, %9 " MI " row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t" \
  "v_fmac_f32_dpp %1, %4, %9 " MI " row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"  \
  "v_fmac_f32_dpp %2, -%11, %15 " MI " row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t" \
  "v_fmac_f32_dpp %3, %10, %15 " MI " row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"  \
  "v_add_f32_e32 %0, %4, %0\n\t"                                               \
  "v_add_f32_e32 %1, %5, %1\n\t"                                               \
  "v_add_f32_e32 %2, %10, %2\n\t"                                               \
  "v_add_f32_e32 %3, %11, %3"

__device__ __forceinline__ void mix3_quad2(cpx& v0, cpx a0, cpx b0, cpx& v1, cpx a1, cpx b1) {
  cpx r0, r1;
  asm(PWFS_MIX3x2_ASM("quad_perm:[1,2,3,0]", "quad_perm:[3,0,1,2]")
      : "=&v"(r0.re), "=&v"(r0.im), "=&v"(r1.re), "=&v"(r1.im)
      : "v"(v0.re), "v"(v0.im), "v"(a0.re), "v"(a0.im), "v"(b0.re), "v"(b0.im),
        "v"(v1.re), "v"(v1.im), "v"(a1.re), "v"(a1.im), "v"(b1.re), "v"(b1.im));
  v0 = r0;
  v1 = r1;
}
#undef PWFS_MIX3x2_ASM

// Row form: v' from lane i + 4 (row_ror:12), v'' from lane i - 4 (row_ror:4),
// mod 16 inside each row of 16 lanes.  Plain DPP moves and FMAs: the long-line
// column pass runs at the 256-register limit, where the early-clobber outputs
// of the DPP-operand form above make the compiler spill.
__device__ __forceinline__ cpx mix3_row4(cpx v, cpx a, cpx b) {
  auto rot = [](float x, auto ctrl) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), decltype(ctrl)::value, 0xF, 0xF, true));
  };
  using P4 = std::integral_constant<int, 0x12C>;
  using M4 = std::integral_constant<int, 0x124>;
  const float pr = rot(v.re, P4{}), pim = rot(v.im, P4{});
  const float nr = rot(v.re, M4{}), nim = rot(v.im, M4{});
  float re = fmaf(a.re, pr, v.re);
  re = fmaf(-a.im, pim, re);
  re = fmaf(b.re, nr, re);
  re = fmaf(-b.im, nim, re);
  float im = fmaf(a.re, pim, v.im);
  im = fmaf(a.im, pr, im);
  im = fmaf(b.re, nim, im);
  im = fmaf(b.im, nr, im);
  return {re, im};
}

// Radix-2 butterfly between the lanes of a quad paired by the DPP pattern PERM
// (0x4E: lane ^ 2, 0xB1: lane ^ 1): self + partner on the lane whose pair bit
// is clear (sgn = +1), partner - self on the other (sgn = -1).
template <int PERM>
__device__ __forceinline__ cpx quad_bfly(cpx v, float sgn) {
  const float pr = quad_perm<PERM>(v.re), pi = quad_perm<PERM>(v.im);
  return {fmaf(sgn, v.re, pr), fmaf(sgn, v.im, pi)};
}
// DFT_4 across the lanes l of a quad, X[k] = sum_l x_l exp(-2 pi i l k / 4),
// decimation in frequency: lane l receives X[rev(l)], rev = (0, 2, 1, 3).
// sA = -1 on lanes with bit 1 set, sB = -1 on lanes with bit 0 set, l3: lane 3.
__device__ __forceinline__ cpx quad_dft4_fwd(cpx v, float sA, float sB, bool l3) {
  cpx u = quad_bfly<0x4E>(v, sA);
  u = l3 ? cpx{u.im, -u.re} : u;  // times -i
  return quad_bfly<0xB1>(u, sB);
}
// Inverse, x_l = sum_k X[k] exp(+2 pi i l k / 4) (no 1/4), from lane l holding
// X[rev(l)] to lane l holding x_l.
__device__ __forceinline__ cpx quad_dft4_inv(cpx v, float sA, float sB, bool l3) {
  cpx p = quad_bfly<0xB1>(v, sB);
  p = l3 ? cpx{-p.im, p.re} : p;  // times +i
  return quad_bfly<0x4E>(p, sA);
}

}  // namespace pwfs
