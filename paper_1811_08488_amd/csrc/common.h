// Device-side building blocks shared by the HIP kernels: storage traits for
// the four field formats, 24-real site loads/stores, link widening and the
// chiral-basis spin projection of the Wilson hop.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace mspcg {

// ---------------------------------------------------------------- storage types
struct bf16 {
  uint16_t bits;
};

template <typename S> struct Traits;
template <> struct Traits<double> {
  using R = double;
  static constexpr bool kNorm = false;
};
template <> struct Traits<float> {
  using R = float;
  static constexpr bool kNorm = false;
};
template <> struct Traits<_Float16> {
  using R = float;
  static constexpr bool kNorm = true;
};
template <> struct Traits<bf16> {
  using R = float;
  static constexpr bool kNorm = true;
};

// bfloat16 <-> float: widening is exact; narrowing rounds to nearest even.
__device__ __host__ inline float bf16_to_float(uint16_t b) {
  union { uint32_t u; float f; } c;
  c.u = (uint32_t)b << 16;
  return c.f;
}
__device__ __host__ inline uint16_t float_to_bf16(float f) {
  union { uint32_t u; float f; } c;
  c.f = f;
  uint32_t u = c.u;
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// ---------------------------------------------------------------- site load/store
// Field layout: the 24 reals of a 5D site are cut into 16-byte chunks (2
// doubles, 4 floats or 8 halves) and the fifth dimension is interleaved
// inside each chunk position:  [rhs][cb][chunk][s][16 bytes].  Lanes that hold
// consecutive s of one 4D site therefore read consecutive 16-byte words with
// every load instruction.  `site4` = rhs * stride + cb counts 4D sites of one
// right-hand side; the per-5D-site norm of F16/BF16 is at site4 * Ls + s.
template <typename S> struct Chunk {
  static constexpr int kReals = 16 / sizeof(S);  // reals per chunk
  static constexpr int kCount = 24 / kReals;     // chunks per 5D site
};
template <typename S>
__device__ __host__ inline size_t chunk_index(size_t site4, int s, int Ls, int c) {
  return ((site4 * Chunk<S>::kCount + c) * (size_t)Ls + s) * Chunk<S>::kReals;
}

template <typename R>
__device__ inline void load24(const double *base, const float *, size_t site4, int s, int Ls, R v[24]) {
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const double2 t = *reinterpret_cast<const double2 *>(base + chunk_index<double>(site4, s, Ls, k));
    v[2 * k] = (R)t.x;
    v[2 * k + 1] = (R)t.y;
  }
}
template <typename R>
__device__ inline void load24(const float *base, const float *, size_t site4, int s, int Ls, R v[24]) {
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const float4 t = *reinterpret_cast<const float4 *>(base + chunk_index<float>(site4, s, Ls, k));
    v[4 * k] = (R)t.x;
    v[4 * k + 1] = (R)t.y;
    v[4 * k + 2] = (R)t.z;
    v[4 * k + 3] = (R)t.w;
  }
}
template <typename R>
__device__ inline void load24(const _Float16 *base, const float *norm, size_t site4, int s, int Ls, R v[24]) {
  const float n = norm[site4 * Ls + s];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const uint4 t = *reinterpret_cast<const uint4 *>(base + chunk_index<_Float16>(site4, s, Ls, k));
    const uint32_t w[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      union { uint32_t u; _Float16 h[2]; } c;
      c.u = w[j];
      v[8 * k + 2 * j] = (R)((float)c.h[0] * n);
      v[8 * k + 2 * j + 1] = (R)((float)c.h[1] * n);
    }
  }
}
template <typename R>
__device__ inline void load24(const bf16 *base, const float *norm, size_t site4, int s, int Ls, R v[24]) {
  const float n = norm[site4 * Ls + s];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const uint4 t = *reinterpret_cast<const uint4 *>(base + chunk_index<bf16>(site4, s, Ls, k));
    const uint32_t w[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      v[8 * k + 2 * j] = (R)(bf16_to_float((uint16_t)(w[j] & 0xffffu)) * n);
      v[8 * k + 2 * j + 1] = (R)(bf16_to_float((uint16_t)(w[j] >> 16)) * n);
    }
  }
}

template <typename R>
__device__ inline void store24(double *base, float *, size_t site4, int s, int Ls, const R v[24]) {
#pragma unroll
  for (int k = 0; k < 12; ++k)
    *reinterpret_cast<double2 *>(base + chunk_index<double>(site4, s, Ls, k)) =
        make_double2((double)v[2 * k], (double)v[2 * k + 1]);
}
template <typename R>
__device__ inline void store24(float *base, float *, size_t site4, int s, int Ls, const R v[24]) {
#pragma unroll
  for (int k = 0; k < 6; ++k)
    *reinterpret_cast<float4 *>(base + chunk_index<float>(site4, s, Ls, k)) =
        make_float4((float)v[4 * k], (float)v[4 * k + 1], (float)v[4 * k + 2], (float)v[4 * k + 3]);
}
template <typename R>
__device__ inline float site_scale(const R v[24], float &inv) {
  float m = 0.f;
#pragma unroll
  for (int k = 0; k < 24; ++k) m = fmaxf(m, fabsf((float)v[k]));
  // (the hardware reciprocal: within one FP32 ulp, far below the 2^-11 or
  // 2^-9 to which the scaled values are then rounded)
  inv = m > 0.f ? __builtin_amdgcn_rcpf(m) : 0.f;
  return m;
}
template <typename R>
__device__ inline void store24(_Float16 *base, float *norm, size_t site4, int s, int Ls, const R v[24]) {
  float inv;
  norm[site4 * Ls + s] = site_scale(v, inv);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    uint32_t w[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      union { uint32_t u; _Float16 h[2]; } c;
      c.h[0] = (_Float16)((float)v[8 * k + 2 * j] * inv);
      c.h[1] = (_Float16)((float)v[8 * k + 2 * j + 1] * inv);
      w[j] = c.u;
    }
    *reinterpret_cast<uint4 *>(base + chunk_index<_Float16>(site4, s, Ls, k)) = make_uint4(w[0], w[1], w[2], w[3]);
  }
}
template <typename R>
__device__ inline void store24(bf16 *base, float *norm, size_t site4, int s, int Ls, const R v[24]) {
  float inv;
  norm[site4 * Ls + s] = site_scale(v, inv);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    uint32_t w[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
      w[j] = (uint32_t)float_to_bf16((float)v[8 * k + 2 * j] * inv) |
             ((uint32_t)float_to_bf16((float)v[8 * k + 2 * j + 1] * inv) << 16);
    *reinterpret_cast<uint4 *>(base + chunk_index<bf16>(site4, s, Ls, k)) = make_uint4(w[0], w[1], w[2], w[3]);
  }
}

// The values a store24 of v followed by a load24 returns, computed in
// registers (F16/BF16: the same per-site scaling and rounding).
template <typename S, typename R>
__device__ inline void stored_values(R v[24]) {
  if constexpr (std::is_same<S, _Float16>::value) {
    float inv;
    const float n = site_scale(v, inv);
#pragma unroll
    for (int k = 0; k < 24; ++k) v[k] = (R)((float)(_Float16)((float)v[k] * inv) * n);
  } else if constexpr (std::is_same<S, bf16>::value) {
    float inv;
    const float n = site_scale(v, inv);
#pragma unroll
    for (int k = 0; k < 24; ++k) v[k] = (R)(bf16_to_float(float_to_bf16((float)v[k] * inv)) * n);
  }
}

// A 5D site as loaded (16-byte chunks, plus the norm for F16/BF16), kept
// raw so that loads can be issued ahead of use and decoded later.
template <typename S> struct RawSite;
template <> struct RawSite<double> {
  double2 c[12];
  __device__ void load(const double *base, const float *, size_t site4, int s, int Ls) {
#pragma unroll
    for (int k = 0; k < 12; ++k) c[k] = *reinterpret_cast<const double2 *>(base + chunk_index<double>(site4, s, Ls, k));
  }
  // p: chunk 0 of the value, cs: the chunk stride (elements)
  __device__ void load_at(const double *p, size_t cs, const float *) {
#pragma unroll
    for (int k = 0; k < 12; ++k) c[k] = *reinterpret_cast<const double2 *>(p + k * cs);
  }
  template <typename R> __device__ void decode(R v[24]) const {
#pragma unroll
    for (int k = 0; k < 12; ++k) { v[2 * k] = (R)c[k].x; v[2 * k + 1] = (R)c[k].y; }
  }
};
template <> struct RawSite<float> {
  float4 c[6];
  __device__ void load(const float *base, const float *, size_t site4, int s, int Ls) {
#pragma unroll
    for (int k = 0; k < 6; ++k) c[k] = *reinterpret_cast<const float4 *>(base + chunk_index<float>(site4, s, Ls, k));
  }
  __device__ void load_at(const float *p, size_t cs, const float *) {
#pragma unroll
    for (int k = 0; k < 6; ++k) c[k] = *reinterpret_cast<const float4 *>(p + k * cs);
  }
  template <typename R> __device__ void decode(R v[24]) const {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      v[4 * k] = (R)c[k].x; v[4 * k + 1] = (R)c[k].y; v[4 * k + 2] = (R)c[k].z; v[4 * k + 3] = (R)c[k].w;
    }
  }
};
template <> struct RawSite<_Float16> {
  uint4 c[3];
  float n;
  __device__ uint32_t word(int i) const { return i < 4 ? (&c[0].x)[i] : i < 8 ? (&c[1].x)[i - 4] : (&c[2].x)[i - 8]; }
  __device__ void set_word(int i, uint32_t w) {
    if (i < 4) (&c[0].x)[i] = w; else if (i < 8) (&c[1].x)[i - 4] = w; else (&c[2].x)[i - 8] = w;
  }
  // the stored values without the norm (each widened once, where it is used)
  __device__ void decode_raw(float v[24]) const {
#pragma unroll
    for (int i = 0; i < 12; ++i) {
      const uint32_t w = word(i);
      union { uint32_t u; _Float16 h[2]; } t;
      t.u = w;
      v[2 * i] = (float)t.h[0];
      v[2 * i + 1] = (float)t.h[1];
    }
  }
  __device__ void load(const _Float16 *base, const float *norm, size_t site4, int s, int Ls) {
    n = norm[site4 * Ls + s];
#pragma unroll
    for (int k = 0; k < 3; ++k) c[k] = *reinterpret_cast<const uint4 *>(base + chunk_index<_Float16>(site4, s, Ls, k));
  }
  __device__ void load_at(const _Float16 *p, size_t cs, const float *np) {
    n = *np;
#pragma unroll
    for (int k = 0; k < 3; ++k) c[k] = *reinterpret_cast<const uint4 *>(p + k * cs);
  }
};
template <> struct RawSite<bf16> {
  uint4 c[3];
  float n;
  __device__ uint32_t word(int i) const { return i < 4 ? (&c[0].x)[i] : i < 8 ? (&c[1].x)[i - 4] : (&c[2].x)[i - 8]; }
  __device__ void set_word(int i, uint32_t w) {
    if (i < 4) (&c[0].x)[i] = w; else if (i < 8) (&c[1].x)[i - 4] = w; else (&c[2].x)[i - 8] = w;
  }
  __device__ void decode_raw(float v[24]) const {
#pragma unroll
    for (int i = 0; i < 12; ++i) {
      const uint32_t w = word(i);
      v[2 * i] = bf16_to_float((uint16_t)(w & 0xffffu));
      v[2 * i + 1] = bf16_to_float((uint16_t)(w >> 16));
    }
  }
  __device__ void load(const bf16 *base, const float *norm, size_t site4, int s, int Ls) {
    n = norm[site4 * Ls + s];
#pragma unroll
    for (int k = 0; k < 3; ++k) c[k] = *reinterpret_cast<const uint4 *>(base + chunk_index<bf16>(site4, s, Ls, k));
  }
  __device__ void load_at(const bf16 *p, size_t cs, const float *np) {
    n = *np;
#pragma unroll
    for (int k = 0; k < 3; ++k) c[k] = *reinterpret_cast<const uint4 *>(p + k * cs);
  }
};

// two halves in one 32-bit register (packed half arithmetic)
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

// An operand that a kernel epilogue combines with its result, kept as stored:
// val(k) is the stored value without the per-site norm (F16/BF16), norm()
// that norm (1 for F64/F32).  The norm then folds into the scalar coefficient
// that multiplies the operand, and for F16 the widening folds into a
// mixed-precision multiply-add.
template <typename S> struct StoredOperand {
  using R = typename Traits<S>::R;
  RawSite<S> raw;
  __device__ void load(const S *base, const float *norm, size_t site4, int s, int Ls) {
    raw.load(base, norm, site4, s, Ls);
  }
  __device__ void zero() { raw = RawSite<S>{}; }
  __device__ R norm() const {
    if constexpr (Traits<S>::kNorm) return raw.n;
    else return R(1);
  }
  __device__ R val(int k) const {
    if constexpr (std::is_same<S, double>::value) {
      return (k & 1) ? raw.c[k >> 1].y : raw.c[k >> 1].x;
    } else if constexpr (std::is_same<S, float>::value) {
      const float4 &c = raw.c[k >> 2];
      return (k & 3) == 0 ? c.x : (k & 3) == 1 ? c.y : (k & 3) == 2 ? c.z : c.w;
    } else if constexpr (std::is_same<S, _Float16>::value) {
      union { uint32_t u; _Float16 h[2]; } t;
      t.u = raw.word(k >> 1);
      return (float)t.h[k & 1];
    } else {
      const uint32_t w = raw.word(k >> 1);
      return bf16_to_float((uint16_t)((k & 1) ? (w >> 16) : (w & 0xffffu)));
    }
  }
};

// store24 that also returns the sum of squares of the values as stored (what
// a load24 would return), for norms of freshly written vectors.  F16: the
// stored halves are squared and summed by packed dot products.
template <typename S, typename R>
__device__ inline R store24_sumsq(S *base, float *norm, size_t site4, int s, int Ls, R v[24]) {
  if constexpr (std::is_same<S, _Float16>::value) {
    float inv;
    const float m = site_scale(v, inv);
    norm[site4 * Ls + s] = m;
    float t = 0.f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      uint32_t w[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        union { uint32_t u; _Float16 h[2]; } c;
        c.h[0] = (_Float16)((float)v[8 * k + 2 * j] * inv);
        c.h[1] = (_Float16)((float)v[8 * k + 2 * j + 1] * inv);
        w[j] = c.u;
        const half2_t h2 = __builtin_bit_cast(half2_t, c.u);
        t = __builtin_amdgcn_fdot2(h2, h2, t, false);
      }
      *reinterpret_cast<uint4 *>(base + chunk_index<_Float16>(site4, s, Ls, k)) = make_uint4(w[0], w[1], w[2], w[3]);
    }
    return t * m * m;
  } else {
    store24<R>(base, norm, site4, s, Ls, v);
    stored_values<S>(v);
    R t = 0;
#pragma unroll
    for (int k = 0; k < 24; ++k) t = fma(v[k], v[k], t);
    return t;
  }
}

// 16 bytes of link data (2 doubles, 4 floats or 8 halves) widened to the compute type.
template <typename R> __device__ inline void widen16(const double *p, R *o) {
  const double2 t = *reinterpret_cast<const double2 *>(p);
  o[0] = (R)t.x; o[1] = (R)t.y;
}
template <typename R> __device__ inline void widen16(const float *p, R *o) {
  const float4 t = *reinterpret_cast<const float4 *>(p);
  o[0] = (R)t.x; o[1] = (R)t.y; o[2] = (R)t.z; o[3] = (R)t.w;
}
template <typename R> __device__ inline void widen16(const _Float16 *p, R *o) {
  const uint4 t = *reinterpret_cast<const uint4 *>(p);
  const uint32_t w[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    union { uint32_t u; _Float16 h[2]; } c;
    c.u = w[j];
    o[2 * j] = (R)(float)c.h[0];
    o[2 * j + 1] = (R)(float)c.h[1];
  }
}
template <typename R> __device__ inline void widen16(const bf16 *p, R *o) {
  const uint4 t = *reinterpret_cast<const uint4 *>(p);
  const uint32_t w[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    o[2 * j] = (R)bf16_to_float((uint16_t)(w[j] & 0xffffu));
    o[2 * j + 1] = (R)bf16_to_float((uint16_t)(w[j] >> 16));
  }
}

// ---------------------------------------------------------------- spin projection
// Chiral basis: g_mu = [[0, B_mu], [B_mu^+, 0]] with B_k = -i sigma_k (k = x,y,z)
// and B_t = 1.  For SGN = +1 the projector is (1 - g_mu), for SGN = -1 it is
// (1 + g_mu).  (1 - SGN g_mu) psi has upper half h = u - SGN B l and lower half
// -SGN B^+ h, so only h (2 spins x 3 colours) is multiplied by the link.
// h = X + Y with X = u (the upper spins) and Y = -SGN B l.
// Indexing: v[(spin*3 + colour)*2 + ri], h[(k*3 + colour)*2 + ri], k = 0,1.
template <int MU, int SGN, typename R>
__device__ inline void project_parts(const R v[24], R X[12], R Y[12]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const R l0r = v[(2 * 3 + c) * 2], l0i = v[(2 * 3 + c) * 2 + 1];
    const R l1r = v[(3 * 3 + c) * 2], l1i = v[(3 * 3 + c) * 2 + 1];
    R y0r, y0i, y1r, y1i;  // -SGN B l
    if (MU == 0) {  // B l = (-i l1, -i l0)
      y0r = -SGN * l1i; y0i = SGN * l1r;
      y1r = -SGN * l0i; y1i = SGN * l0r;
    } else if (MU == 1) {  // B l = (-l1, l0)
      y0r = SGN * l1r; y0i = SGN * l1i;
      y1r = -SGN * l0r; y1i = -SGN * l0i;
    } else if (MU == 2) {  // B l = (-i l0, i l1)
      y0r = -SGN * l0i; y0i = SGN * l0r;
      y1r = SGN * l1i; y1i = -SGN * l1r;
    } else {  // B l = l
      y0r = -SGN * l0r; y0i = -SGN * l0i;
      y1r = -SGN * l1r; y1i = -SGN * l1i;
    }
    X[(0 * 3 + c) * 2] = v[(0 * 3 + c) * 2]; X[(0 * 3 + c) * 2 + 1] = v[(0 * 3 + c) * 2 + 1];
    X[(1 * 3 + c) * 2] = v[(1 * 3 + c) * 2]; X[(1 * 3 + c) * 2 + 1] = v[(1 * 3 + c) * 2 + 1];
    Y[(0 * 3 + c) * 2] = y0r; Y[(0 * 3 + c) * 2 + 1] = y0i;
    Y[(1 * 3 + c) * 2] = y1r; Y[(1 * 3 + c) * 2 + 1] = y1i;
  }
}

template <int MU, int SGN, typename R>
__device__ inline void project(const R v[24], R h[12]) {
  R X[12], Y[12];
  project_parts<MU, SGN>(v, X, Y);
#pragma unroll
  for (int k = 0; k < 12; ++k) h[k] = X[k] + Y[k];
}

// acc += (w, -SGN B^+ w) for one colour c: B_x^+ w = (i w1, i w0),
// B_y^+ w = (w1, -w0), B_z^+ w = (i w0, -i w1), B_t^+ w = (w0, w1).
template <int MU, int SGN, typename R>
__device__ inline void accumulate_colour(R acc[24], int c, R w0r, R w0i, R w1r, R w1i, R n) {
  // acc += n w: n is the per-site norm of F16/BF16 inputs (1 otherwise), so
  // the additions are multiply-adds of the same cost
  acc[(0 * 3 + c) * 2] = fma(n, w0r, acc[(0 * 3 + c) * 2]); acc[(0 * 3 + c) * 2 + 1] = fma(n, w0i, acc[(0 * 3 + c) * 2 + 1]);
  acc[(1 * 3 + c) * 2] = fma(n, w1r, acc[(1 * 3 + c) * 2]); acc[(1 * 3 + c) * 2 + 1] = fma(n, w1i, acc[(1 * 3 + c) * 2 + 1]);
  R l0r, l0i, l1r, l1i;  // -SGN B^+ w
  if (MU == 0) {
    l0r = SGN * w1i; l0i = -SGN * w1r;
    l1r = SGN * w0i; l1i = -SGN * w0r;
  } else if (MU == 1) {
    l0r = -SGN * w1r; l0i = -SGN * w1i;
    l1r = SGN * w0r; l1i = SGN * w0i;
  } else if (MU == 2) {
    l0r = SGN * w0i; l0i = -SGN * w0r;
    l1r = -SGN * w1i; l1i = SGN * w1r;
  } else {
    l0r = -SGN * w0r; l0i = -SGN * w0i;
    l1r = -SGN * w1r; l1i = -SGN * w1i;
  }
  acc[(2 * 3 + c) * 2] = fma(n, l0r, acc[(2 * 3 + c) * 2]); acc[(2 * 3 + c) * 2 + 1] = fma(n, l0i, acc[(2 * 3 + c) * 2 + 1]);
  acc[(3 * 3 + c) * 2] = fma(n, l1r, acc[(3 * 3 + c) * 2]); acc[(3 * 3 + c) * 2 + 1] = fma(n, l1i, acc[(3 * 3 + c) * 2 + 1]);
}

// One direction of the hop for one 5D site, given the projected neighbour
// half spinor h: multiply h by the link U (18 reals, row-major) one colour
// row at a time and add each row's result to both halves of the accumulator
// straight away, so that only the accumulator, the half spinor and one link
// row are live.
template <int MU, int SGN, typename R>
__device__ inline void hop_half(const R h[12], const R *U, R acc[24], R n) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    R ur[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) ur[k] = U[6 * a + k];
    R w[4];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const R *hk = h + 6 * k;
      R re = ur[0] * hk[0];
      R im = ur[0] * hk[1];
      re = fma(-ur[1], hk[1], re);
      im = fma(ur[1], hk[0], im);
#pragma unroll
      for (int b = 1; b < 3; ++b) {
        re = fma(ur[2 * b], hk[2 * b], re);
        re = fma(-ur[2 * b + 1], hk[2 * b + 1], re);
        im = fma(ur[2 * b], hk[2 * b + 1], im);
        im = fma(ur[2 * b + 1], hk[2 * b], im);
      }
      w[2 * k] = re;
      w[2 * k + 1] = im;
    }
    accumulate_colour<MU, SGN>(acc, a, w[0], w[1], w[2], w[3], n);
  }
}

// ---------------------------------------------------------------- FP16 packed projection and link product
// F16 spinors keep each complex component as one 32-bit word (re in the low
// half, im in the high half).  The projection is formed on these pairs with
// packed half-precision adds (the multiplications by +-i and the signs fold
// into the instructions' operand selects and negations), and the link product
// uses two-term dot products of half pairs accumulated in FP32, so that every
// product is exact and every sum is an FP32 sum.  The links of the workgroup
// are staged as pairs A = (re U, -im U), B = (im U, re U) for each complex
// entry: re(U h) = A . h and im(U h) = B . h.

__device__ inline half2_t as_half2(uint32_t w) { return __builtin_bit_cast(half2_t, w); }
__device__ inline half2_t times_i(half2_t z) { return half2_t{-z.y, z.x}; }
template <int SGN> __device__ inline half2_t sgn(half2_t z) { return SGN > 0 ? z : -z; }

// the two parts X (upper spins) and Y = -SGN B l of the projection, as in
// project_parts, on stored words; index k*3 + c for spin k, colour c
template <int MU, int SGN>
__device__ inline void project_parts_h16(const uint32_t w[12], half2_t X[6], half2_t Y[6]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const half2_t l0 = as_half2(w[6 + c]), l1 = as_half2(w[9 + c]);
    X[c] = as_half2(w[c]);
    X[3 + c] = as_half2(w[3 + c]);
    if (MU == 0) {  // B l = (-i l1, -i l0)
      Y[c] = sgn<SGN>(times_i(l1)); Y[3 + c] = sgn<SGN>(times_i(l0));
    } else if (MU == 1) {  // B l = (-l1, l0)
      Y[c] = sgn<SGN>(l1); Y[3 + c] = sgn<-SGN>(l0);
    } else if (MU == 2) {  // B l = (-i l0, i l1)
      Y[c] = sgn<SGN>(times_i(l0)); Y[3 + c] = sgn<-SGN>(times_i(l1));
    } else {  // B l = l
      Y[c] = sgn<-SGN>(l0); Y[3 + c] = sgn<-SGN>(l1);
    }
  }
}

// the link entry pairs (A, B) of one staged 16-byte chunk of F16 links (four
// complex entries) -> eight words
__device__ inline void link_pairs_h16(uint4 q, uint32_t *o) {
  const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    o[2 * j] = w[j] ^ 0x80000000u;          // (re, -im)
    o[2 * j + 1] = (w[j] >> 16) | (w[j] << 16);  // (im, re)
  }
}

// a.x b.x + a.y b.y in FP32 (exact products).  Written as the three-operand
// form with a zero addend: the compiler's own choice for a zero start, the
// accumulating two-operand form, needs a separate move of 0 into the result.
__device__ inline float dot2_from_zero(half2_t a, half2_t b) {
  float r;
  asm("v_dot2_f32_f16 %0, %1, %2, 0" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// hop_half for packed F16 half spinors: acc += n (U h, -SGN B^+ U h), U as
// staged pairs (18 words, row-major), one colour row at a time
template <int MU, int SGN>
__device__ inline void hop_half_h16(const half2_t h[6], const uint32_t *U, float acc[24], float n) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    uint32_t ur[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) ur[k] = U[6 * a + k];
    float w[4];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      float re = dot2_from_zero(as_half2(ur[0]), h[3 * k]);
      float im = dot2_from_zero(as_half2(ur[1]), h[3 * k]);
#pragma unroll
      for (int b = 1; b < 3; ++b) {
        re = __builtin_amdgcn_fdot2(as_half2(ur[2 * b]), h[3 * k + b], re, false);
        im = __builtin_amdgcn_fdot2(as_half2(ur[2 * b + 1]), h[3 * k + b], im, false);
      }
      w[2 * k] = re;
      w[2 * k + 1] = im;
    }
    accumulate_colour<MU, SGN>(acc, a, w[0], w[1], w[2], w[3], n);
  }
}

}  // namespace mspcg
