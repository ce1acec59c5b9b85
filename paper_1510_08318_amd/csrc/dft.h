// In-register complex DFTs for the gfx950 frame transform.
//
// All transforms use the positive exponent, X[k] = sum_n x[n] exp(+2 pi i n k / R),
// unnormalised, natural order in and out (Sec. 3: the image is the Fourier
// transform of the gridded field with the fringe sign of Sec. 2).  Twiddles of
// the in-register stages are compile-time constants; multiplications by 1,
// +-i and the eighth roots are strength-reduced.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace moff {

__device__ __forceinline__ float2 c_add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 c_sub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 c_mul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 c_mul_conj(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 c_mul_i(float2 a) { return make_float2(-a.y, a.x); }
__device__ __forceinline__ float2 c_mul_mi(float2 a) { return make_float2(a.y, -a.x); }
__device__ __forceinline__ float2 c_neg(float2 a) { return make_float2(-a.x, -a.y); }

template <int I, int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// cos / sin of 2 pi k / 16 (k < 16), exact decimal expansions of the
// sixteenth roots of unity.
struct Root16 {
  static constexpr float c1 = 0.92387953251128675613f;  // cos(pi / 8)
  static constexpr float s1 = 0.38268343236508977173f;  // sin(pi / 8)
  static constexpr float r2 = 0.70710678118654752440f;  // sqrt(2) / 2
  static constexpr float re(int k) {
    constexpr float t[16] = {1.f, c1, r2, s1, 0.f, -s1, -r2, -c1, -1.f, -c1, -r2, -s1, 0.f, s1, r2, c1};
    return t[k & 15];
  }
  static constexpr float im(int k) {
    constexpr float t[16] = {0.f, s1, r2, c1, 1.f, c1, r2, s1, 0.f, -s1, -r2, -c1, -1.f, -c1, -r2, -s1};
    return t[k & 15];
  }
};

// a * exp(+2 pi i K16 / 16), 0 <= K16 < 16.
template <int k16>
__device__ __forceinline__ float2 rot16(float2 a) {
  if constexpr (k16 == 0) {
    return a;
  } else if constexpr (k16 == 4) {
    return c_mul_i(a);
  } else if constexpr (k16 == 8) {
    return c_neg(a);
  } else if constexpr (k16 == 12) {
    return c_mul_mi(a);
  } else if constexpr (k16 == 2) {  // (1 + i) / sqrt 2
    return make_float2((a.x - a.y) * Root16::r2, (a.x + a.y) * Root16::r2);
  } else if constexpr (k16 == 6) {  // (-1 + i) / sqrt 2
    return make_float2((-a.x - a.y) * Root16::r2, (a.x - a.y) * Root16::r2);
  } else if constexpr (k16 == 10) {  // (-1 - i) / sqrt 2
    return make_float2((a.y - a.x) * Root16::r2, (-a.x - a.y) * Root16::r2);
  } else if constexpr (k16 == 14) {  // (1 - i) / sqrt 2
    return make_float2((a.x + a.y) * Root16::r2, (a.y - a.x) * Root16::r2);
  } else {
    constexpr float c = Root16::re(k16), s = Root16::im(k16);
    return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
  }
}

// cos / sin of 2 pi k / 32 (k < 32), exact decimal expansions of the
// thirty-second roots of unity; sin(2 pi k / 32) = cos(2 pi (k - 8) / 32).
struct Root32 {
  static constexpr float c1 = 0.98078528040323044913f;  // cos(pi / 16)
  static constexpr float s1 = 0.19509032201612826785f;  // sin(pi / 16)
  static constexpr float c3 = 0.83146961230254523708f;  // cos(3 pi / 16)
  static constexpr float s3 = 0.55557023301960222474f;  // sin(3 pi / 16)
  static constexpr float re(int k) {
    constexpr float t[32] = {1.f,       c1,  Root16::c1,  c3,  Root16::r2,  s3,  Root16::s1,  s1,
                             0.f,       -s1, -Root16::s1, -s3, -Root16::r2, -c3, -Root16::c1, -c1,
                             -1.f,      -c1, -Root16::c1, -c3, -Root16::r2, -s3, -Root16::s1, -s1,
                             0.f,       s1,  Root16::s1,  s3,  Root16::r2,  c3,  Root16::c1,  c1};
    return t[k & 31];
  }
  static constexpr float im(int k) { return re((k - 8) & 31); }
};

// a * exp(+2 pi i K / R), R dividing 32.
template <int R, int K>
__device__ __forceinline__ float2 rot(float2 a) {
  static_assert(32 % R == 0, "rotation order must divide 32");
  constexpr int k = ((K % R) + R) % R;
  constexpr int k32 = k * (32 / R);
  if constexpr (k32 % 2 != 0) {     // an odd thirty-second root
    constexpr float c = Root32::re(k32), s = Root32::im(k32);
    return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
  } else {
    return rot16<k32 / 2>(a);
  }
}

// Dense R-point DFT in registers (R = 1, 2, 4, 8, 16): radix-2 decimation in
// time above a hand-written radix-4 leaf.
template <int R>
struct Dft {
  __device__ __forceinline__ static void run(float2* x) {
    if constexpr (R == 1) {
      return;
    } else if constexpr (R == 2) {
      float2 a = x[0], b = x[1];
      x[0] = c_add(a, b);
      x[1] = c_sub(a, b);
    } else if constexpr (R == 4) {
      float2 s02 = c_add(x[0], x[2]), d02 = c_sub(x[0], x[2]);
      float2 s13 = c_add(x[1], x[3]), d13 = c_mul_i(c_sub(x[1], x[3]));
      x[0] = c_add(s02, s13);
      x[2] = c_sub(s02, s13);
      x[1] = c_add(d02, d13);
      x[3] = c_sub(d02, d13);
    } else {
      float2 e[R / 2], o[R / 2];
#pragma unroll
      for (int m = 0; m < R / 2; ++m) {
        e[m] = x[2 * m];
        o[m] = x[2 * m + 1];
      }
      Dft<R / 2>::run(e);
      Dft<R / 2>::run(o);
      static_for<0, R / 2>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        float2 t = rot<R, k>(o[k]);
        x[k] = c_add(e[k], t);
        x[k + R / 2] = c_sub(e[k], t);
      });
    }
  }
};

// R-point DFT whose inputs x[n] are zero for n >= NZ (NZ a power of two <= R).
// Decimation in frequency removes the zero half:
//   X[2k]   = DFT_{R/2}(x[n])[k],  X[2k+1] = DFT_{R/2}(x[n] w_R^n)[k].
// Only x[0 .. NZ-1] is read.
template <int R, int NZ>
__device__ __forceinline__ void dft_pruned(float2* x) {
  static_assert(NZ >= 1 && NZ <= R && (NZ & (NZ - 1)) == 0, "NZ must be a power of two <= R");
  if constexpr (NZ == R) {
    Dft<R>::run(x);
  } else {
    float2 e[R / 2], o[R / 2];
    static_for<0, NZ>([&](auto nc) {
      constexpr int n = decltype(nc)::value;
      e[n] = x[n];
      o[n] = rot<R, n>(x[n]);
    });
    dft_pruned<R / 2, NZ>(e);
    dft_pruned<R / 2, NZ>(o);
#pragma unroll
    for (int k = 0; k < R / 2; ++k) {
      x[2 * k] = e[k];
      x[2 * k + 1] = o[k];
    }
  }
}

// Inverse-direction R-point DFT, X[k] = sum_n x[n] exp(-2 pi i n k / R), through
// conjugation: conj(DFT(conj(x))).
template <int R>
__device__ __forceinline__ void idft(float2* x) {
#pragma unroll
  for (int i = 0; i < R; ++i) x[i].y = -x[i].y;
  Dft<R>::run(x);
#pragma unroll
  for (int i = 0; i < R; ++i) x[i].y = -x[i].y;
}

}  // namespace moff
