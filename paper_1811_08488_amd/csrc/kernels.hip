// HIP kernels for gfx950: the Ls-fused Wilson hop with fused fifth-dimension
// epilogues, fifth-dimension operators, FP64 BLAS for the outer solver and the
// batched block-CG kernels of the preconditioner.
//
// Thread layout of every site kernel: a workgroup owns `nsite_wg` 4D sites of
// a site list; its threads are (site, rhs, s) with s fastest, so one 4D site's
// Ls x nrhs spinors are handled by consecutive lanes (coalesced loads of the
// [rhs][site][chunk][s] layout, links staged once per site) and the
// fifth-dimension coupling is an exchange between neighbouring lanes (DPP row
// rotation, ds_bpermute or LDS, by the exchange mode below).
#include <algorithm>
#include <type_traits>

#include "common.h"
#include "internal.h"

namespace mspcg {

// ---------------------------------------------------------------- helpers
// Orders a wave's LDS stores before its following LDS loads of words other
// lanes of the same wave stored: wavefront-scope release/acquire fences (the
// compiler neither moves nor forwards memory accesses across them) around a
// wave barrier.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename R>
__device__ inline void zero24(R v[24]) {
#pragma unroll
  for (int k = 0; k < 24; ++k) v[k] = 0;
}

// ---------------------------------------------------------------- fifth-dimension exchange
// The Ls values of one (4D site, rhs) sit on Ls consecutive lanes.  Coupling
// s to s-1 / s+1 is a cyclic rotation inside that group of lanes:
//  * Ls == 16: the group is one DPP row; row_ror moves the value in the same
//    VALU instruction stream, with no LDS traffic and no barrier;
//  * Ls divides 64: groups never straddle a wavefront; ds_bpermute;
//  * otherwise (Ls = 12, 24, ...): through LDS with workgroup barriers.
// (row_ror with all rows and banks enabled writes every lane: no "old" value)
__device__ inline int rot_prev_dpp(int x) { return __builtin_amdgcn_mov_dpp(x, 0x121, 0xF, 0xF, false); }
__device__ inline int rot_next_dpp(int x) { return __builtin_amdgcn_mov_dpp(x, 0x12F, 0xF, 0xF, false); }
__device__ inline float rot_prev_dpp(float x) { return __builtin_bit_cast(float, rot_prev_dpp(__builtin_bit_cast(int, x))); }
__device__ inline float rot_next_dpp(float x) { return __builtin_bit_cast(float, rot_next_dpp(__builtin_bit_cast(int, x))); }
__device__ inline double rot_prev_dpp(double x) {
  const int2 t = __builtin_bit_cast(int2, x);
  return __builtin_bit_cast(double, make_int2(rot_prev_dpp(t.x), rot_prev_dpp(t.y)));
}
__device__ inline double rot_next_dpp(double x) {
  const int2 t = __builtin_bit_cast(int2, x);
  return __builtin_bit_cast(double, make_int2(rot_next_dpp(t.x), rot_next_dpp(t.y)));
}
__device__ inline float perm(int addr, float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(addr, __builtin_bit_cast(int, x)));
}
__device__ inline double perm(int addr, double x) {
  const int2 t = __builtin_bit_cast(int2, x);
  return __builtin_bit_cast(double, make_int2(__builtin_amdgcn_ds_bpermute(addr, t.x), __builtin_amdgcn_ds_bpermute(addr, t.y)));
}

// Exchange modes, fixed per launch from Ls and nrhs (the kernels are
// instantiated per mode), and the lane layout that goes with them.  With DPP
// and ds_bpermute exchanges every 64-lane wave holds G = 64/Ls whole (site,
// rhs) groups of Ls lanes; the last 64 - G*Ls lanes of a wave are idle (4 of
// 64 for Ls = 12).  That layout is used where at most 8 lanes per wave idle
// and some workgroup of whole sites (all nrhs groups of a site together)
// fills whole waves; otherwise (Ls = 24; Ls = 12 with 8 right-hand sides) the
// groups are packed densely and exchange through LDS with barriers.
constexpr int kXDpp16 = 0, kXPerm = 1, kXLds = 2;
// Exchanges through LDS (and the M_5^{-1} transposition) give every thread a
// row of kRow values: the offsets inside a row are instruction immediates, and
// with an odd row length the rows of consecutive threads start on distinct
// banks.
constexpr int kRow = 25;
static inline int xmode(int Ls, int nrhs) {
  if (Ls == 16) return kXDpp16;
  if (Ls > 64) return kXLds;
  const int G = 64 / Ls;
  if (64 % Ls == 0) return kXPerm;
  if (64 - G * Ls > 8) return kXLds;
  for (int c = 1; nrhs * c <= 4 * G; ++c)
    if ((nrhs * c) % G == 0) return kXPerm;
  return kXLds;
}
// groups per wave of the layout (0: dense packing)
__host__ __device__ inline int groups_per_wave(int xm, int Ls) { return xm == kXLds ? 0 : 64 / Ls; }
// thread index of lane t of group g
__device__ inline int group_tid(int G, int Ls, int g, int t) { return G ? (g / G) * 64 + (g % G) * Ls + t : g * Ls + t; }
// threads of a workgroup of `groups` groups
static inline int layout_threads(int xm, int Ls, int groups) {
  const int G = groups_per_wave(xm, Ls);
  return G ? 64 * ((groups + G - 1) / G) : groups * Ls;
}

// v <- a v + b P_chi v (DAG = 0) or a v + b P_chi^+ v (DAG = 1) on the Ls column
// held one s per lane.  P_chi = P- S+ + P+ S-: chirality + (reals 0..11) takes
// s-1, chirality - (reals 12..23) takes s+1, with the -mf corner; the adjoint
// swaps the directions.  Must be reached by all threads of the workgroup.
template <int DAG, int XM, typename R>
__device__ inline void pchi_comb(R *lds, int nthr, int tid, int s, int Ls, R a, R b, R mf, R v[24]) {
  const R cm = (s > 0) ? R(1) : -mf;
  const R cp = (s < Ls - 1) ? R(1) : -mf;
  const R cu = b * (DAG ? cp : cm);
  const R cl = b * (DAG ? cm : cp);
  if (XM == kXDpp16) {
#pragma unroll
    for (int k = 0; k < 12; ++k) v[k] = a * v[k] + cu * (DAG ? rot_next_dpp(v[k]) : rot_prev_dpp(v[k]));
#pragma unroll
    for (int k = 12; k < 24; ++k) v[k] = a * v[k] + cl * (DAG ? rot_prev_dpp(v[k]) : rot_next_dpp(v[k]));
  } else if (XM == kXPerm) {
    const int lane = tid & 63;
    const int am = 4 * ((s > 0) ? lane - 1 : lane + Ls - 1);
    const int ap = 4 * ((s < Ls - 1) ? lane + 1 : lane - (Ls - 1));
    const int au = DAG ? ap : am, al = DAG ? am : ap;
#pragma unroll
    for (int k = 0; k < 12; ++k) v[k] = a * v[k] + cu * perm(au, v[k]);
#pragma unroll
    for (int k = 12; k < 24; ++k) v[k] = a * v[k] + cl * perm(al, v[k]);
  } else {
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 24; ++k) lds[tid * kRow + k] = v[k];
    __syncthreads();
    const int tm = (s > 0) ? tid - 1 : tid + Ls - 1;
    const int tp = (s < Ls - 1) ? tid + 1 : tid - (Ls - 1);
    const int tu = DAG ? tp : tm;
    const int tl = DAG ? tm : tp;
#pragma unroll
    for (int k = 0; k < 12; ++k) v[k] = a * v[k] + cu * lds[tu * kRow + k];
#pragma unroll
    for (int k = 12; k < 24; ++k) v[k] = a * v[k] + cl * lds[tl * kRow + k];
  }
}

// A <- A + P_chi B (DAG = 0) or A + P_chi^+ B (DAG = 1) on the Ls column held one
// s per lane (the directions and corners of pchi_comb): one exchange for a
// combination a u + b P u + c w + d P w of two columns.  Must be reached by
// all threads of the workgroup.
template <int DAG, int XM, typename R>
__device__ inline void pchi_add(R *lds, int nthr, int tid, int s, int Ls, R mf, R A[24], const R B[24]) {
  const R cm = (s > 0) ? R(1) : -mf;
  const R cp = (s < Ls - 1) ? R(1) : -mf;
  const R cu = DAG ? cp : cm;
  const R cl = DAG ? cm : cp;
  if (XM == kXDpp16) {
#pragma unroll
    for (int k = 0; k < 12; ++k) A[k] += cu * (DAG ? rot_next_dpp(B[k]) : rot_prev_dpp(B[k]));
#pragma unroll
    for (int k = 12; k < 24; ++k) A[k] += cl * (DAG ? rot_prev_dpp(B[k]) : rot_next_dpp(B[k]));
  } else if (XM == kXPerm) {
    const int lane = tid & 63;
    const int am = 4 * ((s > 0) ? lane - 1 : lane + Ls - 1);
    const int ap = 4 * ((s < Ls - 1) ? lane + 1 : lane - (Ls - 1));
    const int au = DAG ? ap : am, al = DAG ? am : ap;
#pragma unroll
    for (int k = 0; k < 12; ++k) A[k] += cu * perm(au, B[k]);
#pragma unroll
    for (int k = 12; k < 24; ++k) A[k] += cl * perm(al, B[k]);
  } else {
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 24; ++k) lds[tid * kRow + k] = B[k];
    __syncthreads();
    const int tm = (s > 0) ? tid - 1 : tid + Ls - 1;
    const int tp = (s < Ls - 1) ? tid + 1 : tid - (Ls - 1);
    const int tu = DAG ? tp : tm;
    const int tl = DAG ? tm : tp;
#pragma unroll
    for (int k = 0; k < 12; ++k) A[k] += cu * lds[tu * kRow + k];
#pragma unroll
    for (int k = 12; k < 24; ++k) A[k] += cl * lds[tl * kRow + k];
  }
}

// Projected half spinor of (1 + pc P_chi) v for the hop in direction MU:
// h(s) = X(s) + Y(s) + cu X(s-1) + cl Y(s+1) with X, Y the two parts of the
// projection (P_chi takes the upper spins from s-1 and the lower ones from
// s+1, with the -mf corners folded into cu, cl), so no full M_phi v is formed.
// Must be reached by all threads of the workgroup.
template <int MU, int SGN, int XM, typename R>
__device__ inline void project_pre(R *lds, int nthr, int tid, int s, int Ls, R cu, R cl, const R v[24], R h[12]) {
  // w: the upper spins of v at s-1 and the lower spins at s+1 (rotated raw, so
  // that the signs of the projection fold into the multiply-adds)
  R w[24];
  if (XM == kXDpp16) {
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      w[k] = rot_prev_dpp(v[k]);
      w[12 + k] = rot_next_dpp(v[12 + k]);
    }
  } else if (XM == kXPerm) {
    const int lane = tid & 63;
    const int am = 4 * ((s > 0) ? lane - 1 : lane + Ls - 1);
    const int ap = 4 * ((s < Ls - 1) ? lane + 1 : lane - (Ls - 1));
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      w[k] = perm(am, v[k]);
      w[12 + k] = perm(ap, v[12 + k]);
    }
  } else {
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 24; ++k) lds[tid * kRow + k] = v[k];
    __syncthreads();
    const int tm = (s > 0) ? tid - 1 : tid + Ls - 1;
    const int tp = (s < Ls - 1) ? tid + 1 : tid - (Ls - 1);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      w[k] = lds[tm * kRow + k];
      w[12 + k] = lds[tp * kRow + 12 + k];
    }
  }
  R X[12], Y[12], Xw[12], Yw[12];
  project_parts<MU, SGN>(v, X, Y);
  project_parts<MU, SGN>(w, Xw, Yw);
#pragma unroll
  for (int k = 0; k < 12; ++k) h[k] = fma(cl, Yw[k], fma(cu, Xw[k], X[k] + Y[k]));
}

// wt: the neighbour's weight (1, or 0 outside a block domain; only without M_phi on the input)
template <int MU, int SGN, int PRE, int XM, typename R>
__device__ inline void hop_dir(R *lds, int nthr, int tid, int s, int Ls, R cu, R cl, const R v[24], const R *U,
                               R acc[24], R wt) {
  R h[12];
  if (PRE)
    project_pre<MU, SGN, XM>(lds, nthr, tid, s, Ls, cu, cl, v, h);
  else
    project<MU, SGN>(v, h);
  hop_half<MU, SGN>(h, U, acc, wt);
}

__device__ inline uint32_t rot_prev_word(uint32_t x) { return (uint32_t)rot_prev_dpp((int)x); }
__device__ inline uint32_t rot_next_word(uint32_t x) { return (uint32_t)rot_next_dpp((int)x); }

// The stored words and norm of the upper spins at s-1 and the lower spins at
// s+1 (the part of the neighbouring lanes' inputs that M_phi mixes in).
// Must be reached by all threads of the workgroup.
template <int XM, typename S>
__device__ inline void exchange_pre_raw(float *lds, int nthr, int tid, int s, int Ls, const RawSite<S> &raw,
                                        RawSite<S> &w, float &nm, float &np) {
  if (XM == kXDpp16) {
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      w.set_word(i, rot_prev_word(raw.word(i)));
      w.set_word(6 + i, rot_next_word(raw.word(6 + i)));
    }
    nm = rot_prev_dpp(raw.n);
    np = rot_next_dpp(raw.n);
  } else if (XM == kXPerm) {
    const int lane = tid & 63;
    const int am = 4 * ((s > 0) ? lane - 1 : lane + Ls - 1);
    const int ap = 4 * ((s < Ls - 1) ? lane + 1 : lane - (Ls - 1));
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      w.set_word(i, (uint32_t)__builtin_amdgcn_ds_bpermute(am, (int)raw.word(i)));
      w.set_word(6 + i, (uint32_t)__builtin_amdgcn_ds_bpermute(ap, (int)raw.word(6 + i)));
    }
    nm = perm(am, raw.n);
    np = perm(ap, raw.n);
  } else {
    uint32_t *lw = reinterpret_cast<uint32_t *>(lds);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 12; ++i) lw[tid * kRow + i] = raw.word(i);
    lds[tid * kRow + 12] = raw.n;
    __syncthreads();
    const int tm = (s > 0) ? tid - 1 : tid + Ls - 1;
    const int tp = (s < Ls - 1) ? tid + 1 : tid - (Ls - 1);
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      w.set_word(i, lw[tm * kRow + i]);
      w.set_word(6 + i, lw[tp * kRow + 6 + i]);
    }
    nm = lds[tm * kRow + 12];
    np = lds[tp * kRow + 12];
  }
}

// The same for BF16 inputs stored as v/n with a per-site norm n: the
// projection works on the stored values (widened to FP32) and n multiplies
// the link product as it is accumulated.  With M_phi on the input the
// neighbours' norms enter the mixing coefficients as n(s -+ 1)/n(s) (a zero
// site has no stored values and uses n = 1).  `one` is an opaque 1 that keeps
// each sum a multiply-add.
template <int MU, int SGN, int PRE, int XM, typename S>
__device__ inline void hop_dir_norm(float *lds, int nthr, int tid, int s, int Ls, float cu, float cl, float one,
                                    const RawSite<S> &raw, const float *U, float acc[24], bool out) {
  // every direction widens its own copy of the stored words: shared by the
  // eight direction variants, the widening would be hoisted out of them as
  // separate conversions instead of folding into the multiply-adds
  RawSite<S> rs = raw;
#pragma unroll
  for (int i = 0; i < 12; ++i) {
    uint32_t x = rs.word(i);
    asm volatile("" : "+v"(x));
    rs.set_word(i, x);
  }
  float v[24], X[12], Y[12], h[12];
  rs.decode_raw(v);
  project_parts<MU, SGN>(v, X, Y);
  float n = out ? 0.f : raw.n;
  if (PRE) {
    RawSite<S> w;
    float nm, np;
    exchange_pre_raw<XM>(lds, nthr, tid, s, Ls, raw, w, nm, np);
    float wv[24], Xw[12], Yw[12];
    w.decode_raw(wv);
    project_parts<MU, SGN>(wv, Xw, Yw);
    n = n > 0.f ? n : 1.f;
    const float rn = __builtin_amdgcn_rcpf(n);
    const float cu2 = cu * nm * rn, cl2 = cl * np * rn;
#pragma unroll
    for (int k = 0; k < 12; ++k) h[k] = fmaf(cl2, Yw[k], fmaf(cu2, Xw[k], fmaf(X[k], one, Y[k])));
  } else {
#pragma unroll
    for (int k = 0; k < 12; ++k) h[k] = fmaf(X[k], one, Y[k]);
  }
  hop_half<MU, SGN>(h, U, acc, n);
}

// F16 inputs: the projected half spinor is formed in packed half precision
// on the stored words and multiplied by the link with FP32-accumulated dot
// products (hop_half_h16).  With M_phi on the input the three contributions
// n(s)(X + Y)(s), cu n(s-1) X(s-1) and cl n(s+1) Y(s+1) are scaled by the
// largest of their weights m, so that every coefficient is at most 1 and the
// half-precision sum cannot overflow; m multiplies the link product.
template <int MU, int SGN, int PRE, int XM>
__device__ inline void hop_dir_h16(float *lds, int nthr, int tid, int s, int Ls, float cu, float cl,
                                   const RawSite<_Float16> &raw, const uint32_t *U, float acc[24], bool out) {
  uint32_t wd[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) wd[i] = raw.word(i);
  half2_t X[6], Y[6], h[6];
  project_parts_h16<MU, SGN>(wd, X, Y);
  float m = out ? 0.f : raw.n;
  if (PRE) {
    RawSite<_Float16> w;
    float nm, np;
    exchange_pre_raw<XM>(lds, nthr, tid, s, Ls, raw, w, nm, np);
#pragma unroll
    for (int i = 0; i < 12; ++i) wd[i] = w.word(i);
    half2_t Xw[6], Yw[6];
    project_parts_h16<MU, SGN>(wd, Xw, Yw);
    const float n = raw.n, wu = cu * nm, wl = cl * np;
    m = fmaxf(n, fmaxf(fabsf(wu), fabsf(wl)));
    m = m > 0.f ? m : 1.f;
    const float rm = __builtin_amdgcn_rcpf(m);
    const _Float16 a = (_Float16)(n * rm), bu = (_Float16)(wu * rm), bl = (_Float16)(wl * rm);
#pragma unroll
    for (int k = 0; k < 6; ++k) h[k] = half2_t{a, a} * (X[k] + Y[k]) + (half2_t{bu, bu} * Xw[k] + half2_t{bl, bl} * Yw[k]);
  } else {
#pragma unroll
    for (int k = 0; k < 6; ++k) h[k] = X[k] + Y[k];
  }
  hop_half_h16<MU, SGN>(h, U, acc, m);
}

// ---------------------------------------------------------------- M_5^{-1} along the fifth dimension
// v <- scale X v per chirality for X = sigma (1 + rho S)(1 - q S)^{-1}, S the
// chirality's shift of P_chi (chirality +, reals 0..11: s takes s-1; chirality
// -, reals 12..23: s takes s+1; S^Ls = -mf), or X^T (TR = 1: the shift runs the
// other way).  With sigma = b / alpha, rho = c / b and q = beta / alpha this is
// M_phi M_5^{-1} = (b + c P_chi)(alpha - beta P_chi)^{-1}; with rho = 0 and
// sigma = 1 / alpha it is M_5^{-1} alone (M_5 = alpha - beta P_chi, Eq. (5)).
// Both factors are functions of S, so X v is a first-order recurrence along s
// instead of a dense Ls x Ls product: with positions i counted along the shift
// (i = s, or Ls - 1 - s where the shift takes s+1),
//   u_0 = x_0 + wrap x_{Ls-1},  u_i = x_i + rho x_{i-1}          ((1 + rho S) x)
//   z_0 = u_0,                  z_i = u_i + q z_{i-1}            (no wrap-around)
//   (X x)_i = sigma (z_i + lambda_i z_{Ls-1})
// where wrap = -rho mf and lambda_i = gamma q^i, gamma = -q mf / (1 + mf q^Ls),
// restores the -mf corner of S (exact: (1 - q S)^{-1} = sum_k q^k S^k / (1 + mf q^Ls)).
// cf = [rho, wrap, q, sigma, lambda_0 .. lambda_{Ls-1}] in the compute type.
//
// The Ls values of one (site, rhs) sit on the Ls consecutive threads of its
// group; they are transposed through LDS (rows = positions i, one row of
// kRow words per thread: an odd stride, so a row store of all lanes
// and a column load of all lanes both spread over the banks), lane t of the
// group runs the recurrence of columns t, t + Ls, ... < 24, and the rows are
// read back.  A chirality whose shift takes s+1 is stored with its rows
// reversed, so every column runs toward increasing i.

template <typename R, int LSC>
__device__ inline void chain_columns(R *Tg, int t, int Ls_rt, const R *cf, R sig) {
  const int Ls = LSC > 0 ? LSC : Ls_rt;
  const R rho = cf[0], wrap = cf[1], q = cf[2];
  for (int k = t; k < 24; k += Ls) {
    R *c = Tg + k;
    if constexpr (LSC > 0) {  // the column in registers
      R x[LSC];
#pragma unroll
      for (int i = 0; i < LSC; ++i) x[i] = c[i * kRow];
      R prev = x[0];
      x[0] = fma(wrap, x[LSC - 1], x[0]);
#pragma unroll
      for (int i = 1; i < LSC; ++i) {
        const R cur = x[i];
        x[i] = fma(q, x[i - 1], fma(rho, prev, cur));
        prev = cur;
      }
      const R zl = x[LSC - 1];
#pragma unroll
      for (int i = 0; i < LSC; ++i) c[i * kRow] = sig * fma(cf[4 + i], zl, x[i]);
    } else {  // any Ls: in place in LDS
      R prev = c[0];
      R z = fma(wrap, c[(Ls - 1) * kRow], prev);
      c[0] = z;
      for (int i = 1; i < Ls; ++i) {
        const R cur = c[i * kRow];
        z = fma(q, z, fma(rho, prev, cur));
        c[i * kRow] = z;
        prev = cur;
      }
      for (int i = 0; i < Ls; ++i) c[i * kRow] = sig * fma(cf[4 + i], z, c[i * kRow]);
    }
  }
}

// lds: kRow * nthr values; G: groups per wave of the lane layout (0:
// dense packing, groups may straddle waves: workgroup barriers; otherwise the
// groups of a wave only touch that wave's rows).  Must be reached by all
// threads of the workgroup.
template <int TR, typename R, int LSC>
__device__ inline void m5_chain_t(R *lds, int tid, int s, int Ls_rt, int G, const R *cf, R scale, R v[24]) {
  const int Ls = LSC > 0 ? LSC : Ls_rt;
  R *Tg = lds + (size_t)(tid - s) * kRow;  // this group's rows
  const int rp = TR ? Ls - 1 - s : s;              // row of chirality + (reals 0..11)
  const int rm = TR ? s : Ls - 1 - s;              // row of chirality -
  // The idle lanes past a wave's last whole group (whole-wave layouts) form
  // no group: their rows would run into the next wave's, so they take no part.
  const bool own = G == 0 || ((tid & 63) - s) + Ls <= 64;
  if (G == 0) __syncthreads();                     // (earlier exchanges through the same words)
  if (own) {
#pragma unroll
    for (int k = 0; k < 12; ++k) Tg[rp * kRow + k] = v[k];
#pragma unroll
    for (int k = 12; k < 24; ++k) Tg[rm * kRow + k] = v[k];
  }
  if (G == 0) __syncthreads(); else wave_lds_sync();
  if (own) chain_columns<R, LSC>(Tg, s, Ls, cf, cf[3] * scale);
  if (G == 0) __syncthreads(); else wave_lds_sync();
  if (own) {
#pragma unroll
    for (int k = 0; k < 12; ++k) v[k] = Tg[rp * kRow + k];
#pragma unroll
    for (int k = 12; k < 24; ++k) v[k] = Tg[rm * kRow + k];
  }
}

template <int TR, typename R>
__device__ inline void m5_chain(R *lds, int tid, int s, int Ls, int G, const R *cf, R scale, R v[24]) {
  switch (Ls) {
    case 8: m5_chain_t<TR, R, 8>(lds, tid, s, Ls, G, cf, scale, v); break;
    case 12: m5_chain_t<TR, R, 12>(lds, tid, s, Ls, G, cf, scale, v); break;
    case 16: m5_chain_t<TR, R, 16>(lds, tid, s, Ls, G, cf, scale, v); break;
    case 24: m5_chain_t<TR, R, 24>(lds, tid, s, Ls, G, cf, scale, v); break;
    case 32: m5_chain_t<TR, R, 32>(lds, tid, s, Ls, G, cf, scale, v); break;
    default: m5_chain_t<TR, R, 0>(lds, tid, s, Ls, G, cf, scale, v); break;
  }
}

// Workgroups are dispatched round-robin over the 8 XCDs of the chip, each
// with its own L2.  Renumbering them so that every XCD works on one
// contiguous range of tiles keeps the neighbours a tile gathers (x, y and z
// hops land a few tiles away) in the same L2.  Bijective on [0, n).
__device__ inline int xcd_tile(int b, int n) {
  const int q = n >> 3, rem = n & 7, x = b & 7, k = b >> 3;
  return x * q + min(x, rem) + k;
}

// Workgroup sum of `val` per right-hand side into partial[tile * nrhs + r]
// (fixed order: deterministic).  Uses the LDS region as doubles.
__device__ inline void wg_partial(double *ldsd, int nthr, int tid, int Ls, int nrhs, int nsite_wg, int G, double val,
                                  double *partial, int tile) {
  __syncthreads();
  ldsd[tid] = val;
  __syncthreads();
  const int ngroups = nsite_wg * nrhs;
  if (tid < ngroups) {
    double acc = 0;
    for (int s = 0; s < Ls; ++s) acc += ldsd[group_tid(G, Ls, tid, s)];
    ldsd[nthr + tid] = acc;
  }
  __syncthreads();
  if (tid < nrhs) {
    double acc = 0;
    for (int g = 0; g < nsite_wg; ++g) acc += ldsd[nthr + g * nrhs + tid];
    partial[(size_t)tile * nrhs + tid] = acc;
  }
}

// ---------------------------------------------------------------- the hop kernel
// out(x) = epilogue( sum_mu [ P^{SGN_f}_mu U_mu(x) phi(x+mu) + P^{SGN_b}_mu U_mu(x-mu)^+ phi(x-mu) ] )
// with phi = M_phi in (PRE) or in; SGN_f = +1, SGN_b = -1 for H and the reverse
// for the daggered hop g5 H g5 = H^+.
// Workgroup = (s, rhs, site) threads: threadIdx.x = s, .y = rhs, .z = site.
// GLOBAL: the output list is the whole parity (site_cb a permutation of cb in
// column-sweep order); neighbour tables, outputs and the `other`/dot operands are
// indexed by cb.  Otherwise (block domains) they are indexed by the position
// in the list, and neighbours outside the domain enter with weight zero.
// Occupancy the register allocation of the hop kernel is held to (waves per SIMD).
// (the LDS exchange keeps more values live; FP64 doubles every register)
template <typename S, int XM> struct HopWaves { static constexpr int value = XM == kXLds ? 3 : 4; };
template <int XM> struct HopWaves<double, XM> { static constexpr int value = 2; };
template <int XM> struct HopWaves<float, XM> { static constexpr int value = 3; };  // (FP32 spinors: 4 would spill)

template <typename S, int DAG, int PRE, int EPI, int DOT, int GLOBAL, int XM>
__global__ void __launch_bounds__(256, (HopWaves<S, XM>::value)) hop_kernel(const HopArgs a) {
  using R = typename Traits<S>::R;
  extern __shared__ __align__(16) unsigned char smem[];
  const int Ls = a.Ls, nrhs = a.nrhs, nsw = a.nsite_wg;
  // lane -> (s, group = rhs + nrhs * site-in-workgroup); see groups_per_wave
  const int G = groups_per_wave(XM, Ls);
  const int nthr = blockDim.x * blockDim.y * blockDim.z;
  int s, r, sl, tid;
  bool lane_ok = true;
  if (XM == kXLds) {
    s = threadIdx.x, r = threadIdx.y, sl = threadIdx.z;
    tid = s + Ls * (r + nrhs * sl);
  } else {
    tid = threadIdx.x;
    const int lane = tid & 63, gi = lane / Ls;
    s = lane - gi * Ls;
    int g = (tid >> 6) * G + gi;
    lane_ok = gi < G && g < nrhs * nsw;  // idle lanes compute on the zero site and store nothing
    if (!lane_ok) g = 0;
    r = g % nrhs;
    sl = g / nrhs;
  }
  R *Lk = reinterpret_cast<R *>(smem);  // [nsite_wg][8][18] links of this workgroup's sites
  R *lds = Lk + nsw * 144;              // exchange rows [nthr][kRow] (LDS mode, M_5^{-1})
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int site = tile * nsw + sl;
  const int cbr = (site < a.nsites) ? a.site_cb[site] : -1;
  const bool has_upd = !GLOBAL && a.upd_scal;
  const int ublk = (has_upd && site < a.nsites) ? a.upd_blk[site] : -1;
  const bool active = lane_ok && cbr >= 0;
  const int cb = active ? cbr : 0;
  const int self = GLOBAL ? cb : site;  // index of this site in tables and outputs
  // A fused CG residual update (block domains, upd_scal set) stores
  // out - alpha (result): alpha is requested here, long before it is needed,
  // and -alpha folds into the epilogue's coefficients (all linear in the
  // result).
  const bool upd = has_upd && active;
  double alpha_u = 0;
  if (upd) alpha_u = a.upd_scal[((size_t)ublk * nrhs + r) * kScal + 1];

  // The eight neighbour indices are loaded once, with two 16-byte loads, and
  // kept in registers (rotated by two per direction pair below): no spinor
  // load ever waits for an index load issued after an earlier spinor load.
  // Block domains: a neighbour outside the domain is stored as -1 - n with n
  // an in-domain substitute whose data enters with weight zero (bit d of
  // outm).  Inactive lanes take the neighbours of row 0: they compute on valid
  // data and store nothing.
  int nbw[8];
  int outm = 0;
  {
    const int4 *nb4 = reinterpret_cast<const int4 *>(a.nbr + (size_t)(active ? self : 0) * 8);
    const int4 q0 = nb4[0], q1 = nb4[1];
    const int qa[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
#pragma unroll
    for (int d = 0; d < 8; ++d) {
      if (GLOBAL) {
        nbw[d] = qa[d];
      } else {
        nbw[d] = qa[d] ^ (qa[d] >> 31);  // (-1 - n = ~n)
        outm |= (int)((uint32_t)qa[d] >> 31) << d;
      }
    }
  }
  // the first neighbour spinor is requested before anything else waits
  const S *in = reinterpret_cast<const S *>(a.in);
  const size_t rin = (size_t)r * a.in_stride;
  // neighbour n of this lane: chunk 0 at in_s + n * sstride, its chunks cstride
  // apart, its norm at nrm_s + n * Ls (one multiply-add per address)
  // (32 x 32 -> 64-bit products: one multiply-add each)
  const S *in_s = in + chunk_index<S>(rin, s, Ls, 0);
  const uint32_t cstride = (uint32_t)Ls * Chunk<S>::kReals;
  const uint32_t sstride = cstride * Chunk<S>::kCount;
  const float *nrm_s = Traits<S>::kNorm ? a.in_norm + rin * Ls + s : nullptr;
  auto load_nbr = [&](RawSite<S> &dst, int n) {
    const uint64_t un = (uint32_t)n;
    dst.load_at(in_s + un * sstride, cstride, Traits<S>::kNorm ? nrm_s + un * (uint32_t)Ls : nullptr);
  };
  RawSite<S> cur, nxt;
  load_nbr(cur, nbw[0]);

  // the links of all sites of the workgroup, staged once into LDS with
  // 16-byte loads (every link is used by all Ls x nrhs lanes of its site);
  // the lanes of a site stage that site's links, so no further index is read
  constexpr bool kH16 = std::is_same<S, _Float16>::value;
  if (lane_ok) {
    const S *links = reinterpret_cast<const S *>(a.links);
    constexpr int per = 16 / sizeof(S);
    constexpr int nchunk = 144 / per;
    const S *src = links + (size_t)(cbr >= 0 ? cbr : 0) * 144;
    for (int c = s + Ls * r; c < nchunk; c += Ls * nrhs) {
      if constexpr (kH16)  // F16: (A, B) pairs for the packed link product
        link_pairs_h16(*reinterpret_cast<const uint4 *>(src + c * per),
                       reinterpret_cast<uint32_t *>(Lk) + sl * 144 + c * 8);
      else
        widen16<R>(src + c * per, Lk + sl * 144 + c * per);
    }
  }
  __syncthreads();

  R acc[24];
  zero24(acc);
  const R *Lsite = Lk + sl * 144;
  // PRE: the input is M_phi in = b (1 + (c/b) P_chi) in; the factor b goes
  // into the final scale (handles are created only for b != 0)
  const R pc = PRE ? (R)(a.mphi_c / a.mphi_b) : R(0);
  const R pcu = pc * ((s > 0) ? R(1) : (R)(-a.mf));
  const R pcl = pc * ((s < Ls - 1) ? R(1) : (R)(-a.mf));
  // an opaque 1 (BF16, see hop_dir_norm)
  float one = 1.f;
  asm volatile("" : "+s"(one));
  // One direction is always in flight ahead of the one being computed: the
  // forward neighbour of mu uses buffer `cur`, the backward one `nxt`.  The
  // loop over mu stays rolled on purpose (unrolled, the compiler hoists all
  // eight directions' loads and runs out of registers).
  // FP64 spinors are large: there the register budget is spent on occupancy
  // instead of the prefetch (each direction loads just before it is used).
  constexpr bool kPrefetch = sizeof(R) != 8;
  // (nbw[0], nbw[1]) always hold the indices of directions 2 mu, 2 mu + 1
#pragma unroll 1
  for (int mu = 0; mu < 4; ++mu) {
    if (kPrefetch) load_nbr(nxt, nbw[1]);
#pragma unroll
    for (int bw = 0; bw < 2; ++bw) {
      const int d = 2 * mu + bw;
      // (unconditional: after the last pair nbw[2] is direction 6 again, a
      // cached reload; a load skipped on one path would make the wait
      // before the backward direction drain every load in flight)
      if (kPrefetch && bw == 1) load_nbr(cur, nbw[2]);
      if (!kPrefetch && d > 0) load_nbr(cur, nbw[bw]);
      const R *U = Lsite + d * 18;
      // (1 - g_mu) for the forward hop of H and the backward hop of H^+
      constexpr int sp = (DAG != 0) ? -1 : 1;
      const int sg = bw ? -sp : sp;
      const bool out = !GLOBAL && ((outm >> d) & 1);
#define MSPCG_DIR(M)                                                                                        \
  if constexpr (kH16) {                                                                                     \
    const RawSite<S> &raw = (bw == 0 || !kPrefetch) ? cur : nxt;                                           \
    const uint32_t *Uw = reinterpret_cast<const uint32_t *>(U);                                            \
    if (sg > 0) hop_dir_h16<M, 1, PRE, XM>(lds, nthr, tid, s, Ls, pcu, pcl, raw, Uw, acc, out);             \
    else hop_dir_h16<M, -1, PRE, XM>(lds, nthr, tid, s, Ls, pcu, pcl, raw, Uw, acc, out);                   \
  } else if constexpr (Traits<S>::kNorm) {                                                                  \
    const RawSite<S> &raw = (bw == 0 || !kPrefetch) ? cur : nxt;                                           \
    if (sg > 0) hop_dir_norm<M, 1, PRE, XM>(lds, nthr, tid, s, Ls, pcu, pcl, one, raw, U, acc, out);        \
    else hop_dir_norm<M, -1, PRE, XM>(lds, nthr, tid, s, Ls, pcu, pcl, one, raw, U, acc, out);              \
  } else {                                                                                                  \
    R v[24];                                                                                                \
    if (bw == 0 || !kPrefetch) cur.decode(v); else nxt.decode(v);                                           \
    const R wt = out ? R(0) : R(1);                                                                         \
    if (sg > 0) hop_dir<M, 1, PRE, XM>(lds, nthr, tid, s, Ls, pcu, pcl, v, U, acc, wt);                     \
    else hop_dir<M, -1, PRE, XM>(lds, nthr, tid, s, Ls, pcu, pcl, v, U, acc, wt);                           \
  }
      switch (mu) {
        case 0: MSPCG_DIR(0) break;
        case 1: MSPCG_DIR(1) break;
        case 2: MSPCG_DIR(2) break;
        default: MSPCG_DIR(3) break;
      }
#undef MSPCG_DIR
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) nbw[k] = nbw[k + 2];
  }

  const R scale = (R)(PRE ? a.scale * a.mphi_b : a.scale);
  // (the opaque copy keeps the conversion, and so the wait for the load, here)
  asm volatile("" : "+v"(alpha_u));
  const R fu = upd ? -(R)alpha_u : R(1);
  if (EPI == EPI_M5INV) {
    m5_chain<DAG, R>(lds, tid, s, Ls, G, reinterpret_cast<const R *>(a.mat), scale, acc);
  } else if (EPI == EPI_MPHIDAG) {
    pchi_comb<1, XM, R>(lds, nthr, tid, s, Ls, (R)a.mphi_b, (R)a.mphi_c, (R)a.mf, acc);
#pragma unroll
    for (int k = 0; k < 24; ++k) acc[k] *= scale;
  } else if (EPI == EPI_SCALE) {
#pragma unroll
    for (int k = 0; k < 24; ++k) acc[k] *= scale;
  }
  if (EPI == EPI_M5_OTHER || EPI == EPI_M5DAG_MPHIDAG) {
    // (outside the block domain the operand vanishes; those lanes load
    // nothing: a shared substitute site would draw the reads of every such
    // lane onto one cache line)
    const int oi = GLOBAL ? cb : (active ? (a.other_idx ? a.other_idx[site] : site) : -1);
    StoredOperand<S> o;
    o.zero();
    if (oi >= 0) o.load(reinterpret_cast<const S *>(a.other), a.other_norm, (size_t)r * a.other_stride + oi, s, Ls);
    const R ow = oi >= 0 ? o.norm() * fu : R(0);
    // M_5 = alpha - beta P_chi, M_5^+ = alpha - beta P_chi^+, M_phi^+ = b + c P_chi^+:
    //   M_5 o + scale h                 = (alpha o + scale h) + P_chi (-beta o)
    //   M_5^+ o + scale M_phi^+ h       = (alpha o + scale b h) + P_chi^+ (-beta o + scale c h)
    // (every coefficient times fu; the operand's norm with those of o)
    const R al = (R)a.m5_alpha * ow, mbe = (R)(-a.m5_beta) * ow;
    const R sb = (EPI == EPI_M5DAG_MPHIDAG ? scale * (R)a.mphi_b : scale) * fu;
    const R sc = (R)a.mphi_c * scale * fu;
    R B[24];
#pragma unroll
    for (int k = 0; k < 24; ++k) {
      const R ok = o.val(k);
      B[k] = EPI == EPI_M5DAG_MPHIDAG ? fma(ok, mbe, sc * acc[k]) : ok * mbe;
      acc[k] = fma(ok, al, sb * acc[k]);
    }
    pchi_add<EPI == EPI_M5DAG_MPHIDAG ? 1 : 0, XM, R>(lds, nthr, tid, s, Ls, (R)a.mf, acc, B);
  } else if (upd) {
#pragma unroll
    for (int k = 0; k < 24; ++k) acc[k] *= fu;
  }

  R sumsq = 0;  // |out|^2 of the values as stored (DOT after a fused update)
  if (upd) {  // out <- out - alpha (result), read in place
    StoredOperand<S> ro;
    ro.load(reinterpret_cast<const S *>(a.out), a.out_norm, (size_t)r * a.out_stride + self, s, Ls);
    const R rn = ro.norm();
#pragma unroll
    for (int k = 0; k < 24; ++k) acc[k] = fma(ro.val(k), rn, acc[k]);
    if (DOT && !a.dotw)
      sumsq = store24_sumsq<S, R>(reinterpret_cast<S *>(a.out), a.out_norm, (size_t)r * a.out_stride + self, s, Ls,
                                  acc);
    else
      store24<R>(reinterpret_cast<S *>(a.out), a.out_norm, (size_t)r * a.out_stride + self, s, Ls, acc);
  } else if (active) {
    store24<R>(reinterpret_cast<S *>(a.out), a.out_norm, (size_t)r * a.out_stride + self, s, Ls, acc);
  }

  if (DOT) {  // Re<w, out>, or |out|^2 without w (of the values as stored, after a fused update)
    double val = 0;
    if (active) {
      R t = 0;
      if (a.dotw) {
        R w[24];
        load24<R>(reinterpret_cast<const S *>(a.dotw), a.dotw_norm, (size_t)r * a.dotw_stride + self, s, Ls, w);
#pragma unroll
        for (int k = 0; k < 24; ++k) t += w[k] * acc[k];
      } else if (upd) {
        t = sumsq;
      } else {
#pragma unroll
        for (int k = 0; k < 24; ++k) t += acc[k] * acc[k];
      }
      val = (double)t;
    }
    wg_partial(reinterpret_cast<double *>(smem), nthr, tid, Ls, nrhs, nsw, G, val, a.partial, tile);
  }
}

template <typename S>
static size_t hop_lds_bytes(const HopArgs &a, int nthr, int epi, int dot, int xm) {
  using R = typename Traits<S>::R;
  size_t b = (size_t)144 * a.nsite_wg * sizeof(R);
  if (epi == EPI_M5INV || xm == kXLds) b += (size_t)kRow * nthr * sizeof(R);
  if (dot) b = std::max(b, (size_t)2 * nthr * sizeof(double));
  return b;
}

template <typename S, int DAG, int PRE, int EPI, int DOT, int GLOBAL>
static hipError_t launch_hop_t(const HopArgs &a, hipStream_t st) {
  const int xm = xmode(a.Ls, a.nrhs);
  const int nthr = layout_threads(xm, a.Ls, a.nsite_wg * a.nrhs);
  const int grid = (a.nsites + a.nsite_wg - 1) / a.nsite_wg;
  if (a.nsite_wg < 1 || nthr > 256 || grid < 1) return hipErrorInvalidValue;
  const dim3 blk = (xm == kXLds) ? dim3(a.Ls, a.nrhs, a.nsite_wg) : dim3(nthr);
  const size_t lds = hop_lds_bytes<S>(a, nthr, EPI, DOT, xm);
  switch (xm) {
    case kXDpp16: hipLaunchKernelGGL((hop_kernel<S, DAG, PRE, EPI, DOT, GLOBAL, kXDpp16>), dim3(grid), blk, lds, st, a); break;
    case kXPerm: hipLaunchKernelGGL((hop_kernel<S, DAG, PRE, EPI, DOT, GLOBAL, kXPerm>), dim3(grid), blk, lds, st, a); break;
    default: hipLaunchKernelGGL((hop_kernel<S, DAG, PRE, EPI, DOT, GLOBAL, kXLds>), dim3(grid), blk, lds, st, a); break;
  }
  return hipGetLastError();
}

int hop_threads(int Ls, int nrhs, int nsite_wg) { return layout_threads(xmode(Ls, nrhs), Ls, nrhs * nsite_wg); }
int hop_groups_per_wave(int Ls, int nrhs) { return groups_per_wave(xmode(Ls, nrhs), Ls); }

template <typename S>
static hipError_t dispatch_hop(int dagger, int pre, int epi, int dot, int global, const HopArgs &a, hipStream_t st) {
  // the combinations used by the operators (anything else is rejected)
#define MSPCG_HOP(D, P, E, T, G)                                                \
  if (dagger == D && pre == P && epi == E && dot == T && (global != 0) == (G != 0)) \
    return launch_hop_t<S, D, P, E, T, G>(a, st);
  MSPCG_HOP(0, 1, EPI_SCALE, 0, 1)          // M^4 in
  MSPCG_HOP(1, 0, EPI_MPHIDAG, 0, 1)        // (M^4)^+ in
  MSPCG_HOP(0, 1, EPI_M5INV, 0, 1)          // M_phi M_5^-1 M^4 in (first hop of D_PC)
  MSPCG_HOP(0, 0, EPI_M5_OTHER, 0, 1)       // M_5 psi + 1/2 H c
  MSPCG_HOP(1, 0, EPI_M5INV, 0, 1)          // M_5^-+ M_phi^+ (M^4)^+ y
  MSPCG_HOP(1, 0, EPI_M5DAG_MPHIDAG, 0, 1)  // M_5^+ y + 1/2 M_phi^+ H^+ f
  MSPCG_HOP(1, 0, EPI_M5DAG_MPHIDAG, 1, 1)  //   ... with the fused <w, out>
  MSPCG_HOP(0, 0, EPI_M5INV, 0, 0)          // the same four hops on block domains (M_phi p formed beforehand;
                                            // neighbours outside a domain enter with weight zero, which needs
                                            // the input unmixed: no M_phi on the input there)
  MSPCG_HOP(0, 0, EPI_M5_OTHER, 0, 0)
  MSPCG_HOP(0, 0, EPI_M5_OTHER, 1, 0)          //   ... with the fused |out|^2 (<p, A_s p> = |D_PC P_s p|^2)
  MSPCG_HOP(1, 0, EPI_M5INV, 0, 0)
  MSPCG_HOP(1, 0, EPI_M5DAG_MPHIDAG, 0, 0)
  MSPCG_HOP(1, 0, EPI_M5DAG_MPHIDAG, 1, 0)
#undef MSPCG_HOP
  return hipErrorInvalidValue;
}

hipError_t launch_hop(int prec, int dagger, int pre, int epi, int dot, int global, const HopArgs &a, hipStream_t st) {
  switch (prec) {
    case MSPCG_F64: return dispatch_hop<double>(dagger, pre, epi, dot, global, a, st);
    case MSPCG_F32: return dispatch_hop<float>(dagger, pre, epi, dot, global, a, st);
    case MSPCG_F16: return dispatch_hop<_Float16>(dagger, pre, epi, dot, global, a, st);
    case MSPCG_BF16: return dispatch_hop<bf16>(dagger, pre, epi, dot, global, a, st);
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------- fifth-dimension operator
template <typename S, int XM>
__global__ void __launch_bounds__(256) op5_kernel(const Op5Args a) {
  using R = typename Traits<S>::R;
  extern __shared__ __align__(16) unsigned char smem[];
  const int Ls = a.Ls, nrhs = a.nrhs;
  const int G = groups_per_wave(XM, Ls);  // lane layout as in hop_kernel
  const int nthr = blockDim.x * blockDim.y * blockDim.z;
  int s, r, sl, tid;
  bool lane_ok = true;
  if (XM == kXLds) {
    s = threadIdx.x, r = threadIdx.y, sl = threadIdx.z;
    tid = s + Ls * (r + nrhs * sl);
  } else {
    tid = threadIdx.x;
    const int lane = tid & 63, gi = lane / Ls;
    s = lane - gi * Ls;
    int g = (tid >> 6) * G + gi;
    lane_ok = gi < G && g < nrhs * a.nsite_wg;
    if (!lane_ok) g = 0;
    r = g % nrhs;
    sl = g / nrhs;
  }
  R *lds = reinterpret_cast<R *>(smem);
  const int site = blockIdx.x * a.nsite_wg + sl;
  const bool active = lane_ok && site < a.nsites;
  R v[24];
  const size_t idx = (size_t)r * a.stride + (active ? site : 0);
  load24<R>(reinterpret_cast<const S *>(a.in), a.in_norm, idx, s, Ls, v);
  if (a.inv && a.dag)
    m5_chain<1, R>(lds, tid, s, Ls, G, reinterpret_cast<const R *>(a.chain), R(1), v);
  else if (a.inv)
    m5_chain<0, R>(lds, tid, s, Ls, G, reinterpret_cast<const R *>(a.chain), R(1), v);
  else if (a.dag)
    pchi_comb<1, XM, R>(lds, nthr, tid, s, Ls, (R)a.a, (R)a.b, (R)a.mf, v);
  else
    pchi_comb<0, XM, R>(lds, nthr, tid, s, Ls, (R)a.a, (R)a.b, (R)a.mf, v);
  if (active) store24<R>(reinterpret_cast<S *>(a.out), a.out_norm, idx, s, Ls, v);
}

template <typename S>
static void launch_op5_t(const Op5Args &a, dim3 grid, dim3 blk, size_t lds, hipStream_t st) {
  switch (xmode(a.Ls, a.nrhs)) {
    case kXDpp16: hipLaunchKernelGGL((op5_kernel<S, kXDpp16>), grid, blk, lds, st, a); break;
    case kXPerm: hipLaunchKernelGGL((op5_kernel<S, kXPerm>), grid, blk, lds, st, a); break;
    default: hipLaunchKernelGGL((op5_kernel<S, kXLds>), grid, blk, lds, st, a); break;
  }
}

hipError_t launch_op5(int prec, const Op5Args &a, hipStream_t st) {
  const int xm = xmode(a.Ls, a.nrhs);
  const int nthr = layout_threads(xm, a.Ls, a.nsite_wg * a.nrhs);
  const int grid = (a.nsites + a.nsite_wg - 1) / a.nsite_wg;
  if (a.nsite_wg < 1 || nthr > 256 || grid < 1) return hipErrorInvalidValue;
  const size_t rsz = (prec == MSPCG_F64) ? 8 : 4;
  const size_t lds = (size_t)kRow * nthr * rsz;
  const dim3 blk = (xm == kXLds) ? dim3(a.Ls, a.nrhs, a.nsite_wg) : dim3(nthr);
  switch (prec) {
    case MSPCG_F64: launch_op5_t<double>(a, dim3(grid), blk, lds, st); break;
    case MSPCG_F32: launch_op5_t<float>(a, dim3(grid), blk, lds, st); break;
    case MSPCG_F16: launch_op5_t<_Float16>(a, dim3(grid), blk, lds, st); break;
    case MSPCG_BF16: launch_op5_t<bf16>(a, dim3(grid), blk, lds, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- conversion
template <typename SO, typename SI>
__global__ void convert_kernel(SO *out, float *out_norm, const SI *in, const float *in_norm, long long n5, int Ls) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n5) return;
  const size_t site4 = (size_t)(i / Ls);
  const int s = (int)(i % Ls);
  if (sizeof(SI) == 8 || sizeof(SO) == 8) {
    double t[24];
    load24<double>(in, in_norm, site4, s, Ls, t);
    store24<double>(out, out_norm, site4, s, Ls, t);
  } else {
    float v[24];
    load24<float>(in, in_norm, site4, s, Ls, v);
    store24<float>(out, out_norm, site4, s, Ls, v);
  }
}

template <typename SO>
static hipError_t convert_from(const Vec &out, const Vec &in, long long n5, int Ls, hipStream_t st) {
  const int blk = 256;
  const long long grid = (n5 + blk - 1) / blk;
  SO *o = reinterpret_cast<SO *>(out.data);
  switch (in.prec) {
    case MSPCG_F64: hipLaunchKernelGGL((convert_kernel<SO, double>), dim3(grid), dim3(blk), 0, st, o, out.norm, (const double *)in.data, in.norm, n5, Ls); break;
    case MSPCG_F32: hipLaunchKernelGGL((convert_kernel<SO, float>), dim3(grid), dim3(blk), 0, st, o, out.norm, (const float *)in.data, in.norm, n5, Ls); break;
    case MSPCG_F16: hipLaunchKernelGGL((convert_kernel<SO, _Float16>), dim3(grid), dim3(blk), 0, st, o, out.norm, (const _Float16 *)in.data, in.norm, n5, Ls); break;
    case MSPCG_BF16: hipLaunchKernelGGL((convert_kernel<SO, bf16>), dim3(grid), dim3(blk), 0, st, o, out.norm, (const bf16 *)in.data, in.norm, n5, Ls); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_convert(const Vec &out, const Vec &in, int nrhs, long long nsites5, int Ls, hipStream_t st) {
  const long long n5 = nsites5 * nrhs;
  if (n5 <= 0) return hipSuccess;
  switch (out.prec) {
    case MSPCG_F64: return convert_from<double>(out, in, n5, Ls, st);
    case MSPCG_F32: return convert_from<float>(out, in, n5, Ls, st);
    case MSPCG_F16: return convert_from<_Float16>(out, in, n5, Ls, st);
    case MSPCG_BF16: return convert_from<bf16>(out, in, n5, Ls, st);
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------- FP64 BLAS
// Grid (kBlasGrid, nrhs) with a grid-stride loop over double2 pairs: the set
// of elements each thread sums, and the reduction tree, depend only on n.
__device__ inline void block_sum_store(double v, double *out) {
  __shared__ double sh[kBlasWG];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = kBlasWG / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

__global__ void __launch_bounds__(kBlasWG) k_dot(const double *a, const double *b, long long n, double *partial) {
  const int r = blockIdx.y;
  const double2 *x = reinterpret_cast<const double2 *>(a + (size_t)r * n);
  const double2 *y = reinterpret_cast<const double2 *>(b + (size_t)r * n);
  const long long n2 = n / 2;
  double acc = 0;
  for (long long i = (long long)blockIdx.x * kBlasWG + threadIdx.x; i < n2; i += (long long)kBlasGrid * kBlasWG) {
    const double2 u = x[i], v = y[i];
    acc += u.x * v.x + u.y * v.y;
  }
  block_sum_store(acc, partial + (size_t)blockIdx.x * gridDim.y + r);
}

hipError_t blas_dot_partial(const double *a, const double *b, long long n, int nrhs, double *partial, hipStream_t st) {
  hipLaunchKernelGGL(k_dot, dim3(kBlasGrid, nrhs), dim3(kBlasWG), 0, st, a, b, n, partial);
  return hipGetLastError();
}

// partial[p][r] -> out[r]; one workgroup per right-hand side
__global__ void __launch_bounds__(kBlasWG) k_reduce(const double *partial, int nparts, int nrhs, double *out) {
  const int r = blockIdx.x;
  double acc = 0;
  for (int p = threadIdx.x; p < nparts; p += kBlasWG) acc += partial[(size_t)p * nrhs + r];
  block_sum_store(acc, out + r);
}

hipError_t blas_reduce(const double *partial, int nparts, int nrhs, double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce, dim3(nrhs), dim3(kBlasWG), 0, st, partial, nparts, nrhs, out);
  return hipGetLastError();
}

__global__ void __launch_bounds__(kBlasWG) k_update_xr(double *xv, double *rv, const double *pv, const double *qv,
                                                       const double *alpha, long long n, double *partial) {
  const int r = blockIdx.y;
  const double al = alpha[r];
  double2 *x = reinterpret_cast<double2 *>(xv + (size_t)r * n);
  double2 *rr = reinterpret_cast<double2 *>(rv + (size_t)r * n);
  const double2 *p = reinterpret_cast<const double2 *>(pv + (size_t)r * n);
  const double2 *q = reinterpret_cast<const double2 *>(qv + (size_t)r * n);
  const long long n2 = n / 2;
  double acc = 0;
  for (long long i = (long long)blockIdx.x * kBlasWG + threadIdx.x; i < n2; i += (long long)kBlasGrid * kBlasWG) {
    double2 xi = x[i], ri = rr[i];
    const double2 pi = p[i], qi = q[i];
    xi.x += al * pi.x; xi.y += al * pi.y;
    ri.x -= al * qi.x; ri.y -= al * qi.y;
    x[i] = xi;
    rr[i] = ri;
    acc += ri.x * ri.x + ri.y * ri.y;
  }
  block_sum_store(acc, partial + (size_t)blockIdx.x * gridDim.y + r);
}

hipError_t blas_update_xr(double *x, double *r, const double *p, const double *q, const double *alpha, long long n,
                          int nrhs, double *partial, hipStream_t st) {
  hipLaunchKernelGGL(k_update_xr, dim3(kBlasGrid, nrhs), dim3(kBlasWG), 0, st, x, r, p, q, alpha, n, partial);
  return hipGetLastError();
}

__global__ void __launch_bounds__(kBlasWG) k_xpay(double *pv, const double *zv, const double *beta, long long n) {
  const int r = blockIdx.y;
  const double be = beta[r];
  double2 *p = reinterpret_cast<double2 *>(pv + (size_t)r * n);
  const double2 *z = reinterpret_cast<const double2 *>(zv + (size_t)r * n);
  const long long n2 = n / 2;
  for (long long i = (long long)blockIdx.x * kBlasWG + threadIdx.x; i < n2; i += (long long)kBlasGrid * kBlasWG) {
    double2 pi = p[i];
    const double2 zi = z[i];
    pi.x = zi.x + be * pi.x;
    pi.y = zi.y + be * pi.y;
    p[i] = pi;
  }
}

hipError_t blas_xpay(double *p, const double *z, const double *beta, long long n, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(k_xpay, dim3(kBlasGrid, nrhs), dim3(kBlasWG), 0, st, p, z, beta, n);
  return hipGetLastError();
}

__global__ void __launch_bounds__(kBlasWG) k_axpby(double *ov, double a, const double *xv, double b, const double *yv,
                                                   long long n) {
  const int r = blockIdx.y;
  double2 *o = reinterpret_cast<double2 *>(ov + (size_t)r * n);
  const double2 *x = reinterpret_cast<const double2 *>(xv + (size_t)r * n);
  const double2 *y = reinterpret_cast<const double2 *>(yv + (size_t)r * n);
  const long long n2 = n / 2;
  for (long long i = (long long)blockIdx.x * kBlasWG + threadIdx.x; i < n2; i += (long long)kBlasGrid * kBlasWG) {
    const double2 xi = x[i], yi = y[i];
    o[i] = make_double2(a * xi.x + b * yi.x, a * xi.y + b * yi.y);
  }
}

hipError_t blas_axpby(double *out, double a, const double *x, double b, const double *y, long long n, int nrhs,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_axpby, dim3(kBlasGrid, nrhs), dim3(kBlasWG), 0, st, out, a, x, b, y, n);
  return hipGetLastError();
}

__global__ void k_solver_scalars(int mode, int nrhs, const int *active, double *rho, const double *x1, double *out,
                                 const double *x2, const double *x3) {
  const int r = threadIdx.x;
  if (r >= nrhs) return;
  const bool on = active[r] != 0;
  if (mode == 0) {
    const double pap = x1[r];
    out[r] = (on && pap != 0.0) ? rho[r] / pap : 0.0;
  } else if (mode == 1) {
    const double rn = x1[r];
    out[r] = (on && rho[r] != 0.0) ? rn / rho[r] : 0.0;
    if (on) rho[r] = rn;
  } else {
    const double rn = x1[r], zq = x2[r], pap = x3[r];
    out[r] = (on && pap != 0.0) ? -zq / pap : 0.0;
    if (on) rho[r] = rn;
  }
}

hipError_t solver_scalars(int mode, int nrhs, const int *active, double *rho, const double *x1, double *out,
                          hipStream_t st, const double *x2, const double *x3) {
  if (mode == 2 && (!x2 || !x3)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_solver_scalars, dim3(1), dim3(64), 0, st, mode, nrhs, active, rho, x1, out, x2, x3);
  return hipGetLastError();
}

// ---------------------------------------------------------------- block preconditioner
// The B_e list is ordered block by block, each block padded to a multiple of
// 64 sites, so with nsite_wg dividing 64 every workgroup lies in one block.
// M_phi v = b v + c P_chi v for the Ls values of one (site, rhs) held on
// consecutive threads of a block kernel (layout tid = s + Ls (rhs + nrhs site)),
// exchanged through LDS; all threads of the workgroup must reach it.
template <typename R>
__device__ inline void block_mphi(R *lds, int nthr, int tid, int s, int Ls, const BlockArgs &b, R v[24]) {
  pchi_comb<0, kXLds, R>(lds, nthr, tid, s, Ls, (R)b.mphi_b, (R)b.mphi_c, (R)b.mf, v);
}

template <typename S>
__global__ void __launch_bounds__(256) k_block_gather(const BlockArgs b, Vec xs, Vec rs, Vec ps, Vec mps,
                                                       const double *rg, long long rg_stride, const double *rr,
                                                       double n_total, double *partial) {
  using R = typename Traits<S>::R;
  extern __shared__ __align__(16) unsigned char smem[];
  const int nthr = blockDim.x, tid = threadIdx.x, Ls = b.Ls, G = b.nrhs * Ls;
  const int sl = tid / G, rem = tid - sl * G, r = rem / Ls, s = rem - r * Ls;
  const int site = blockIdx.x * b.nsite_wg + sl;
  const int cb = site < b.nsites ? b.be_cb[site] : -1;
  const size_t o = (size_t)r * rs.stride + site;
  double val = 0;
  R v[24];
  zero24(v);
  if (cb >= 0) {
    const double scale = rr ? (rr[r] > 0 ? sqrt(n_total / rr[r]) : 0.0) : 1.0;
    double t[24];
    load24<double>(rg, nullptr, (size_t)r * rg_stride + cb, s, Ls, t);
#pragma unroll
    for (int k = 0; k < 24; ++k) v[k] = (R)(scale * t[k]);
    store24<R>(reinterpret_cast<S *>(rs.data), rs.norm, o, s, Ls, v);
    // the values as stored, so that r and p start identical and the sum matches them
    stored_values<S>(v);
    store24<R>(reinterpret_cast<S *>(ps.data), ps.norm, o, s, Ls, v);
    if (xs.data) {  // (the fixed-k solve sets x in its first update instead)
      R z[24];
      zero24(z);
      store24<R>(reinterpret_cast<S *>(xs.data), xs.norm, o, s, Ls, z);
    }
    R acc = 0;
#pragma unroll
    for (int k = 0; k < 24; ++k) acc += v[k] * v[k];
    val = (double)acc;
  }
  block_mphi<R>(reinterpret_cast<R *>(smem), nthr, tid, s, Ls, b, v);
  if (cb >= 0) store24<R>(reinterpret_cast<S *>(mps.data), mps.norm, o, s, Ls, v);
  wg_partial(reinterpret_cast<double *>(smem), nthr, tid, Ls, b.nrhs, b.nsite_wg, 0, val, partial, blockIdx.x);
}

template <typename S>
__global__ void __launch_bounds__(256) k_block_scatter(const BlockArgs b, double *zg, long long zg_stride, Vec xs,
                                                        Vec ps, const double *scal, int mode, const double *rg,
                                                        long long rg_stride, const double *rr, double n_total,
                                                        double *partial) {
  using R = typename Traits<S>::R;
  extern __shared__ __align__(16) unsigned char smem[];
  const int nthr = blockDim.x, tid = threadIdx.x, Ls = b.Ls, G = b.nrhs * Ls;
  const int sl = tid / G, rem = tid - sl * G, r = rem / Ls, s = rem - r * Ls;
  const int site = blockIdx.x * b.nsite_wg + sl;
  const int cb = site < b.nsites ? b.be_cb[site] : -1;
  double val = 0;
  if (cb >= 0) {
    const double inv = rr ? (rr[r] > 0 ? sqrt(rr[r] / n_total) : 0.0) : 1.0;
    const size_t o = (size_t)r * xs.stride + site;
    R v[24];
    if (mode == 2) zero24(v); else load24<R>(reinterpret_cast<const S *>(xs.data), xs.norm, o, s, Ls, v);
    if (mode != 0) {  // the last inner iteration's x update, not stored: x + alpha p
      const int blk = b.be_blk[site];
      const R al = (R)scal[((size_t)blk * b.nrhs + r) * kScal + 1];
      R pv[24];
      load24<R>(reinterpret_cast<const S *>(ps.data), ps.norm, o, s, Ls, pv);
#pragma unroll
      for (int k = 0; k < 24; ++k) v[k] = fma(al, pv[k], v[k]);
    }
    double z[24], t[24];
#pragma unroll
    for (int k = 0; k < 24; ++k) z[k] = inv * (double)v[k];
    if (zg) store24<double>(zg, nullptr, (size_t)r * zg_stride + cb, s, Ls, z);  // (none: only the partials)
    if (rg) {
      load24<double>(rg, nullptr, (size_t)r * rg_stride + cb, s, Ls, t);
#pragma unroll
      for (int k = 0; k < 24; ++k) val += z[k] * t[k];
    }
  }
  wg_partial(reinterpret_cast<double *>(smem), nthr, tid, Ls, b.nrhs, b.nsite_wg, 0, val, partial, blockIdx.x);
}

// The outer direction update fused with the scatter: p(cb) = v / scale +
// beta p(cb) (first: p = v / scale) with v as in k_block_scatter, so the
// preconditioned residual z is never stored.
template <typename S>
__global__ void __launch_bounds__(256) k_block_scatter_xpay(const BlockArgs b, double *pg, long long pg_stride, Vec xs,
                                                             Vec ps, const double *scal, int mode, const double *rr,
                                                             double n_total, const double *beta, int first) {
  using R = typename Traits<S>::R;
  const int tid = threadIdx.x, Ls = b.Ls, G = b.nrhs * Ls;
  const int sl = tid / G, rem = tid - sl * G, r = rem / Ls, s = rem - r * Ls;
  const int site = blockIdx.x * b.nsite_wg + sl;
  const int cb = site < b.nsites ? b.be_cb[site] : -1;
  if (cb < 0) return;
  const double inv = rr ? (rr[r] > 0 ? sqrt(rr[r] / n_total) : 0.0) : 1.0;
  const size_t o = (size_t)r * xs.stride + site;
  R v[24];
  if (mode == 2) zero24(v); else load24<R>(reinterpret_cast<const S *>(xs.data), xs.norm, o, s, Ls, v);
  if (mode != 0) {
    const R al = (R)scal[((size_t)b.be_blk[site] * b.nrhs + r) * kScal + 1];
    R pv[24];
    load24<R>(reinterpret_cast<const S *>(ps.data), ps.norm, o, s, Ls, pv);
#pragma unroll
    for (int k = 0; k < 24; ++k) v[k] = fma(al, pv[k], v[k]);
  }
  const size_t g = (size_t)r * pg_stride + cb;
  double pn[24];
  if (first) {
#pragma unroll
    for (int k = 0; k < 24; ++k) pn[k] = inv * (double)v[k];
  } else {
    load24<double>(pg, nullptr, g, s, Ls, pn);
    const double be = beta[r];
#pragma unroll
    for (int k = 0; k < 24; ++k) pn[k] = fma(be, pn[k], inv * (double)v[k]);
  }
  store24<double>(pg, nullptr, g, s, Ls, pn);
}

template <typename S>
__global__ void __launch_bounds__(256) k_block_update_xr(const BlockArgs b, Vec xv, Vec rv, Vec pv, Vec qv,
                                                          const double *scal, double *partial) {
  using R = typename Traits<S>::R;
  extern __shared__ __align__(16) unsigned char smem[];
  const int nthr = blockDim.x, tid = threadIdx.x, Ls = b.Ls, G = b.nrhs * Ls;
  const int sl = tid / G, rem = tid - sl * G, r = rem / Ls, s = rem - r * Ls;
  const int site = blockIdx.x * b.nsite_wg + sl;
  const int blk = site < b.nsites ? b.be_blk[site] : -1;
  double val = 0;
  if (blk >= 0) {
    const R al = (R)scal[((size_t)blk * b.nrhs + r) * kScal + 1];
    const size_t o = (size_t)r * xv.stride + site;
    R x[24], rr[24], p[24], q[24];
    load24<R>(reinterpret_cast<const S *>(xv.data), xv.norm, o, s, Ls, x);
    load24<R>(reinterpret_cast<const S *>(rv.data), rv.norm, o, s, Ls, rr);
    load24<R>(reinterpret_cast<const S *>(pv.data), pv.norm, o, s, Ls, p);
    load24<R>(reinterpret_cast<const S *>(qv.data), qv.norm, o, s, Ls, q);
#pragma unroll
    for (int k = 0; k < 24; ++k) {
      x[k] += al * p[k];
      rr[k] -= al * q[k];
    }
    store24<R>(reinterpret_cast<S *>(xv.data), xv.norm, o, s, Ls, x);
    store24<R>(reinterpret_cast<S *>(rv.data), rv.norm, o, s, Ls, rr);
    // the norm is taken of the stored (rounded) residual
    stored_values<S>(rr);
    R acc = 0;
#pragma unroll
    for (int k = 0; k < 24; ++k) acc += rr[k] * rr[k];
    val = (double)acc;
  }
  wg_partial(reinterpret_cast<double *>(smem), nthr, tid, Ls, b.nrhs, b.nsite_wg, 0, val, partial, blockIdx.x);
}

// r -= alpha Ap with the partial |r|^2 (every iteration but the last, where
// k_block_update_xr also updates x)
template <typename S>
__global__ void __launch_bounds__(256) k_block_update_r(const BlockArgs b, Vec rv, Vec qv, const double *scal,
                                                        double *partial) {
  using R = typename Traits<S>::R;
  extern __shared__ __align__(16) unsigned char smem[];
  const int nthr = blockDim.x, tid = threadIdx.x, Ls = b.Ls, G = b.nrhs * Ls;
  const int sl = tid / G, rem = tid - sl * G, r = rem / Ls, s = rem - r * Ls;
  const int site = blockIdx.x * b.nsite_wg + sl;
  const int blk = site < b.nsites ? b.be_blk[site] : -1;
  double val = 0;
  if (blk >= 0) {
    const R al = (R)scal[((size_t)blk * b.nrhs + r) * kScal + 1];
    const size_t o = (size_t)r * rv.stride + site;
    R rr[24], q[24];
    load24<R>(reinterpret_cast<const S *>(rv.data), rv.norm, o, s, Ls, rr);
    load24<R>(reinterpret_cast<const S *>(qv.data), qv.norm, o, s, Ls, q);
#pragma unroll
    for (int k = 0; k < 24; ++k) rr[k] -= al * q[k];
    store24<R>(reinterpret_cast<S *>(rv.data), rv.norm, o, s, Ls, rr);
    stored_values<S>(rr);
    R acc = 0;
#pragma unroll
    for (int k = 0; k < 24; ++k) acc += rr[k] * rr[k];
    val = (double)acc;
  }
  wg_partial(reinterpret_cast<double *>(smem), nthr, tid, Ls, b.nrhs, b.nsite_wg, 0, val, partial, blockIdx.x);
}

// x += alpha p, then p = r + beta p (the x update of k_block_update_xr moved
// here, where p is read anyway), and M_phi p for the next first hop (from the
// values as stored)
template <typename S>
__global__ void __launch_bounds__(256) k_block_update_xp(const BlockArgs b, Vec xv, Vec pv, Vec mpv, Vec rv,
                                                         const double *scal, int first) {
  using R = typename Traits<S>::R;
  extern __shared__ __align__(16) unsigned char smem[];
  const int nthr = blockDim.x, tid = threadIdx.x, Ls = b.Ls, G = b.nrhs * Ls;
  const int sl = tid / G, rem = tid - sl * G, r = rem / Ls, s = rem - r * Ls;
  const int site = blockIdx.x * b.nsite_wg + sl;
  const int blk = site < b.nsites ? b.be_blk[site] : -1;
  const size_t o = (size_t)r * pv.stride + site;
  R p[24];
  zero24(p);
  if (blk >= 0) {
    const double *sc = scal + ((size_t)blk * b.nrhs + r) * kScal;
    const R al = (R)sc[1], be = (R)sc[2];
    R x[24], rr[24];
    if (first) zero24(x);  // (x_0 = 0: not read)
    else load24<R>(reinterpret_cast<const S *>(xv.data), xv.norm, o, s, Ls, x);
    load24<R>(reinterpret_cast<const S *>(pv.data), pv.norm, o, s, Ls, p);
    load24<R>(reinterpret_cast<const S *>(rv.data), rv.norm, o, s, Ls, rr);
#pragma unroll
    for (int k = 0; k < 24; ++k) {
      x[k] += al * p[k];
      p[k] = rr[k] + be * p[k];
    }
    store24<R>(reinterpret_cast<S *>(xv.data), xv.norm, o, s, Ls, x);
    store24<R>(reinterpret_cast<S *>(pv.data), pv.norm, o, s, Ls, p);
    stored_values<S>(p);
  }
  block_mphi<R>(reinterpret_cast<R *>(smem), nthr, tid, s, Ls, b, p);
  if (blk >= 0) store24<R>(reinterpret_cast<S *>(mpv.data), mpv.norm, o, s, Ls, p);
}

// one workgroup per (block, rhs): a fixed-shape tree sum of that block's
// workgroup partials (deterministic), then the CG scalar update
__global__ void __launch_bounds__(256) k_block_scalars(int mode, int nrhs, int nsite_wg, const int *be_off,
                                                       const double *partial, double *scal) {
  __shared__ double sh[256];
  const int blk = blockIdx.x, r = blockIdx.y;
  const int w0 = be_off[blk] / nsite_wg, w1 = be_off[blk + 1] / nsite_wg;
  double sum = 0;
  for (int w = w0 + (int)threadIdx.x; w < w1; w += 256) sum += partial[(size_t)w * nrhs + r];
  sh[threadIdx.x] = sum;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  sum = sh[0];
  double *sc = scal + ((size_t)blk * nrhs + r) * kScal;
  if (mode == 0) {
    sc[1] = (sum > 0.0 && sc[0] > 0.0) ? sc[0] / sum : 0.0;
  } else if (mode == 1) {
    sc[2] = (sc[0] > 0.0) ? sum / sc[0] : 0.0;
    sc[0] = sum;
  } else {
    sc[0] = sum;
    sc[1] = sc[2] = 0.0;
  }
}

static inline int block_threads(const BlockArgs &b) { return b.nsite_wg * b.nrhs * b.Ls; }
static inline int block_grid(const BlockArgs &b) { return (b.nsites + b.nsite_wg - 1) / b.nsite_wg; }
static inline size_t block_lds(const BlockArgs &b) { return (size_t)2 * block_threads(b) * sizeof(double); }
// the kernels that form M_phi p exchange 24 reals per thread through LDS
template <typename S>
static inline size_t block_lds_mphi(const BlockArgs &b) {
  return std::max(block_lds(b), (size_t)kRow * block_threads(b) * sizeof(typename Traits<S>::R));
}

#define MSPCG_PREC_SWITCH(prec, CALL)                 \
  switch (prec) {                                     \
    case MSPCG_F64: { using S = double; CALL; } break;   \
    case MSPCG_F32: { using S = float; CALL; } break;    \
    case MSPCG_F16: { using S = _Float16; CALL; } break; \
    case MSPCG_BF16: { using S = bf16; CALL; } break;    \
    default: return hipErrorInvalidValue;             \
  }

hipError_t block_gather(int prec, const BlockArgs &b, const Vec &xs, const Vec &rs, const Vec &ps, const Vec &mps,
                        const Vec &rglob, const double *rr, double n_total, double *partial, hipStream_t st) {
  if (rglob.prec != MSPCG_F64 || block_threads(b) > 256) return hipErrorInvalidValue;
  MSPCG_PREC_SWITCH(prec, hipLaunchKernelGGL(k_block_gather<S>, dim3(block_grid(b)), dim3(block_threads(b)),
                                             block_lds_mphi<S>(b), st, b, xs, rs, ps, mps,
                                             (const double *)rglob.data, rglob.stride, rr, n_total, partial));
  return hipGetLastError();
}

hipError_t block_scatter(int prec, const BlockArgs &b, const Vec &zglob, const Vec &xs, const Vec &ps,
                         const double *scal, int mode, const Vec &rglob, const double *rr, double n_total,
                         double *partial, hipStream_t st) {
  if (zglob.prec != MSPCG_F64 || block_threads(b) > 256 || mode < 0 || mode > 2) return hipErrorInvalidValue;
  MSPCG_PREC_SWITCH(prec, hipLaunchKernelGGL(k_block_scatter<S>, dim3(block_grid(b)), dim3(block_threads(b)),
                                             block_lds(b), st, b, (double *)zglob.data, zglob.stride, xs, ps, scal,
                                             mode, (const double *)rglob.data, rglob.stride, rr, n_total, partial));
  return hipGetLastError();
}

hipError_t block_scatter_xpay(int prec, const BlockArgs &b, const Vec &pglob, const Vec &xs, const Vec &ps,
                              const double *scal, int mode, const double *rr, double n_total, const double *beta,
                              int first, hipStream_t st) {
  if (pglob.prec != MSPCG_F64 || block_threads(b) > 256 || mode < 0 || mode > 2) return hipErrorInvalidValue;
  MSPCG_PREC_SWITCH(prec, hipLaunchKernelGGL(k_block_scatter_xpay<S>, dim3(block_grid(b)), dim3(block_threads(b)), 0,
                                             st, b, (double *)pglob.data, pglob.stride, xs, ps, scal, mode, rr,
                                             n_total, beta, first));
  return hipGetLastError();
}

hipError_t block_scalars(int mode, const BlockArgs &b, const double *partial, double *scal, hipStream_t st) {
  const int n = b.nblocks * b.nrhs;
  (void)n;
  hipLaunchKernelGGL(k_block_scalars, dim3(b.nblocks, b.nrhs), dim3(256), 0, st, mode, b.nrhs, b.nsite_wg, b.be_off,
                     partial, scal);
  return hipGetLastError();
}

hipError_t block_update_xr(int prec, const BlockArgs &b, const Vec &x, const Vec &r, const Vec &p, const Vec &Ap,
                           const double *scal, double *partial, hipStream_t st) {
  if (block_threads(b) > 256) return hipErrorInvalidValue;
  MSPCG_PREC_SWITCH(prec, hipLaunchKernelGGL(k_block_update_xr<S>, dim3(block_grid(b)), dim3(block_threads(b)),
                                             block_lds(b), st, b, x, r, p, Ap, scal, partial));
  return hipGetLastError();
}

hipError_t block_update_r(int prec, const BlockArgs &b, const Vec &r, const Vec &Ap, const double *scal,
                          double *partial, hipStream_t st) {
  if (block_threads(b) > 256) return hipErrorInvalidValue;
  MSPCG_PREC_SWITCH(prec, hipLaunchKernelGGL(k_block_update_r<S>, dim3(block_grid(b)), dim3(block_threads(b)),
                                             block_lds(b), st, b, r, Ap, scal, partial));
  return hipGetLastError();
}

hipError_t block_update_xp(int prec, const BlockArgs &b, const Vec &x, const Vec &p, const Vec &mp, const Vec &r,
                           const double *scal, int first, hipStream_t st) {
  if (block_threads(b) > 256) return hipErrorInvalidValue;
  MSPCG_PREC_SWITCH(prec, hipLaunchKernelGGL(k_block_update_xp<S>, dim3(block_grid(b)), dim3(block_threads(b)),
                                             block_lds_mphi<S>(b), st, b, x, p, mp, r, scal, first));
  return hipGetLastError();
}

// ---------------------------------------------------------------- link packing
template <typename S>
__global__ void k_pack_links(S *out, const double *gauge, const int *lex_of_cb, const int *nbr_lex, int Vh, int Lt,
                             int Lxyz, double tbc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;  // (cb, d)
  if (i >= Vh * 8) return;
  const int cb = i >> 3, d = i & 7, mu = d >> 1, bw = d & 1;
  const int x = lex_of_cb[cb];
  const int t = x / Lxyz;
  const int src = bw ? nbr_lex[(size_t)cb * 8 + d] : x;
  const double sign = (mu == 3 && ((!bw && t == Lt - 1) || (bw && t == 0))) ? tbc : 1.0;
  const double *U = gauge + ((size_t)src * 4 + mu) * 18;
  S *o = out + (size_t)i * 18;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double re, im;
      if (!bw) { re = U[(a * 3 + b) * 2]; im = U[(a * 3 + b) * 2 + 1]; }
      else { re = U[(b * 3 + a) * 2]; im = -U[(b * 3 + a) * 2 + 1]; }
      re *= sign;
      im *= sign;
      if constexpr (std::is_same<S, bf16>::value) {
        o[(a * 3 + b) * 2].bits = float_to_bf16((float)re);
        o[(a * 3 + b) * 2 + 1].bits = float_to_bf16((float)im);
      } else {
        o[(a * 3 + b) * 2] = (S)re;
        o[(a * 3 + b) * 2 + 1] = (S)im;
      }
    }
}

hipError_t pack_links(int prec, void *out, const double *gauge, const int *lex_of_cb, const int *nbr_lex, int parity,
                      int Vh, int Lt, int Lxyz, double tbc, hipStream_t st) {
  (void)parity;
  const int n = Vh * 8, blk = 256;
  MSPCG_PREC_SWITCH(prec, hipLaunchKernelGGL(k_pack_links<S>, dim3((n + blk - 1) / blk), dim3(blk), 0, st,
                                             reinterpret_cast<S *>(out), gauge, lex_of_cb, nbr_lex, Vh, Lt, Lxyz, tbc));
  return hipGetLastError();
}

}  // namespace mspcg
