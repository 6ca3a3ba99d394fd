// FP64 CPU oracle for the multisplitting-preconditioned CG (MSPCG) solve of the
// even-odd preconditioned Moebius domain-wall-fermion (DWF) Dirac equation.
//
// TEST INFRASTRUCTURE ONLY.  This file is the slow, literal reference that the
// GPU library is checked against.  Only the test suite, the smoke check and the
// benchmark's CPU-baseline leg may load it; the product path never does.  It
// shares no code, header, table or helper with the GPU library.
//
// Everything here follows the definitions step by step, in FP64, on
// full-lattice fields in lexicographic order:
//   * 4D sites: lex = x + Lx*(y + Ly*(z + Lz*t)), parity = (x+y+z+t) mod 2
//     (Sec. 2.2, definition of the even/odd parity).
//   * A 5D fermion field is psi[lex][s][spin][colour] (complex).
//   * The gauge field is U[lex][mu][row][col] (complex), mu = x,y,z,t.
//   * Antiperiodic (or periodic) time: a hop that crosses between t=Lt-1 and
//     t=0 picks up the factor tbc; the links themselves are not modified.
//
// Readings where the paper defers or is garbled (all fixed as project
// conventions, shared with the GPU library only through this documentation):
//   * Wilson hop (Sec. 2.2, definition of D^w, printed with a dagger on both
//     links): read as the gauge-covariant
//       H psi(x) = sum_mu [ (1-g_mu) U_mu(x) psi(x+mu) + (1+g_mu) U_mu(x-mu)^+ psi(x-mu) ]
//     with D^w == -1/2 H, i.e. D_W(-M5) = (4-M5) - H/2.
//   * Moebius 5th dimension (Sec. 2.2 defers to Brower et al.):
//       (S+ v)(s) = v(s+1), (S+ v)(Ls-1) = -mf v(0)
//       (S- v)(s) = v(s-1), (S- v)(0)    = -mf v(Ls-1)
//       P_chi = P- S+ + P+ S-,  P+- = (1 +- g5)/2
//       M_phi = b + c P_chi
//       D     = D_W (b + c P_chi) + (1 - P_chi)
//     so the site-diagonal block is M_5 = (4-M5) M_phi + 1 - P_chi and the
//     hopping block is M^4 = -1/2 H M_phi.
//   * Chiral gamma basis: g_k = [[0,-i s_k],[i s_k,0]] (k = x,y,z),
//     g_t = [[0,1],[1,0]], g5 = g_x g_y g_z g_t = diag(1,1,-1,-1).
//
// Parity-packed ("cb") fields used at this file's C interface: one parity p,
// [cb][s][spin][colour][re,im] with cb = lex >> 1 for the sites of parity p.

#include <complex>
#include <vector>
#include <cmath>
#include <cstring>
#include <cstdint>
#include <omp.h>

typedef std::complex<double> cplx;
typedef std::vector<cplx> Field;

namespace {

// ---------------------------------------------------------------- parameters
struct Params {
  int L[4];
  int V;
  int Ls;
  double M5, mf, b, c, tbc;
};

bool make_params(const int *L, int Ls, const double *p, Params &P) {
  if (!L || !p || Ls < 2) return false;
  P.V = 1;
  for (int mu = 0; mu < 4; ++mu) {
    if (L[mu] < 2 || (L[mu] & 1)) return false;
    P.L[mu] = L[mu];
    P.V *= L[mu];
  }
  P.Ls = Ls;
  P.M5 = p[0]; P.mf = p[1]; P.b = p[2]; P.c = p[3]; P.tbc = p[4];
  return true;
}

// ---------------------------------------------------------------- geometry
// Sec. 2.2: parity = (x+y+z+t) mod 2.
void coords(const Params &P, int lex, int c[4]) {
  for (int mu = 0; mu < 4; ++mu) { c[mu] = lex % P.L[mu]; lex /= P.L[mu]; }
}
int lex_of(const Params &P, const int c[4]) {
  return c[0] + P.L[0] * (c[1] + P.L[1] * (c[2] + P.L[2] * c[3]));
}
int parity_of(const Params &P, int lex) {
  int c[4]; coords(P, lex, c);
  return (c[0] + c[1] + c[2] + c[3]) % 2;
}
// neighbour x + dir*mu (periodic wrap); *phase gets the time boundary factor
int neighbour(const Params &P, int lex, int mu, int dir, double *phase) {
  int c[4]; coords(P, lex, c);
  int v = c[mu] + dir;
  double ph = 1.0;
  if (v == P.L[mu]) { v = 0; if (mu == 3) ph = P.tbc; }
  if (v < 0) { v = P.L[mu] - 1; if (mu == 3) ph = P.tbc; }
  c[mu] = v;
  if (phase) *phase = ph;
  return lex_of(P, c);
}

// Blocks (Sec. 2.1 fig. 1, Sec. 2.4: one block of sites per processor).  Block
// j of n along a dimension of extent L starts at j*floor(L/n) + min(j, L mod n)
// and has floor(L/n) + [j < L mod n] sites.  Block id = jx + nx(jy + ny(jz + nz jt)).
int block_coord(int x, int L, int n) {
  for (int j = 0; j < n; ++j) {
    int start = j * (L / n) + (j < L % n ? j : L % n);
    int size = L / n + (j < L % n ? 1 : 0);
    if (x >= start && x < start + size) return j;
  }
  return -1;
}
int block_of(const Params &P, const int *nblk, int lex) {
  int c[4]; coords(P, lex, c);
  int id = 0;
  for (int mu = 3; mu >= 0; --mu) id = id * nblk[mu] + block_coord(c[mu], P.L[mu], nblk[mu]);
  return id;
}

// ---------------------------------------------------------------- spin algebra
typedef cplx Mat4[4][4];

struct Gammas {
  Mat4 g[4];    // g_x, g_y, g_z, g_t
  Mat4 g5;
  Mat4 one_minus[4], one_plus[4];  // 1 - g_mu, 1 + g_mu
  Mat4 Pplus, Pminus;              // (1 +- g5)/2
};

void matmul4(const Mat4 a, const Mat4 b, Mat4 out) {
  Mat4 t;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      cplx acc = 0;
      for (int k = 0; k < 4; ++k) acc += a[i][k] * b[k][j];
      t[i][j] = acc;
    }
  std::memcpy(out, t, sizeof(Mat4));
}

Gammas make_gammas() {
  const cplx I(0, 1);
  // Pauli matrices
  cplx s[3][2][2] = {{{0, 1}, {1, 0}}, {{0, -I}, {I, 0}}, {{1, 0}, {0, -1}}};
  Gammas G;
  for (int mu = 0; mu < 4; ++mu)
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) G.g[mu][i][j] = 0;
  for (int k = 0; k < 3; ++k)
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) {
        G.g[k][i][2 + j] = -I * s[k][i][j];
        G.g[k][2 + i][j] = I * s[k][i][j];
      }
  for (int i = 0; i < 2; ++i) { G.g[3][i][2 + i] = 1; G.g[3][2 + i][i] = 1; }
  Mat4 t;
  matmul4(G.g[0], G.g[1], t);
  matmul4(t, G.g[2], t);
  matmul4(t, G.g[3], G.g5);
  for (int mu = 0; mu < 4; ++mu)
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) {
        cplx id = (i == j) ? 1.0 : 0.0;
        G.one_minus[mu][i][j] = id - G.g[mu][i][j];
        G.one_plus[mu][i][j] = id + G.g[mu][i][j];
      }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      cplx id = (i == j) ? 1.0 : 0.0;
      G.Pplus[i][j] = 0.5 * (id + G.g5[i][j]);
      G.Pminus[i][j] = 0.5 * (id - G.g5[i][j]);
    }
  return G;
}

const Gammas &gammas() {
  static const Gammas G = make_gammas();
  return G;
}

// ---------------------------------------------------------------- 5th dimension
// A 5D-local operator acts identically on every 4D site and colour; it is a
// dense (4 Ls) x (4 Ls) complex matrix on the (s, spin) index i = 4 s + spin.
struct Op5 {
  int n = 0;
  std::vector<cplx> m;  // row-major n x n
  cplx &at(int i, int j) { return m[(size_t)i * n + j]; }
  cplx at(int i, int j) const { return m[(size_t)i * n + j]; }
};

Op5 op5_zero(int n) { Op5 o; o.n = n; o.m.assign((size_t)n * n, 0.0); return o; }
Op5 op5_identity(int n) { Op5 o = op5_zero(n); for (int i = 0; i < n; ++i) o.at(i, i) = 1; return o; }
Op5 op5_lincomb(cplx a, const Op5 &A, cplx b, const Op5 &B) {
  Op5 o = op5_zero(A.n);
  for (size_t k = 0; k < o.m.size(); ++k) o.m[k] = a * A.m[k] + b * B.m[k];
  return o;
}
Op5 op5_dagger(const Op5 &A) {
  Op5 o = op5_zero(A.n);
  for (int i = 0; i < A.n; ++i)
    for (int j = 0; j < A.n; ++j) o.at(i, j) = std::conj(A.at(j, i));
  return o;
}
// Gauss-Jordan inverse with partial pivoting.
Op5 op5_inverse(const Op5 &A) {
  int n = A.n;
  Op5 a = A, inv = op5_identity(n);
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (std::abs(a.at(r, col)) > std::abs(a.at(piv, col))) piv = r;
    for (int j = 0; j < n; ++j) {
      std::swap(a.at(col, j), a.at(piv, j));
      std::swap(inv.at(col, j), inv.at(piv, j));
    }
    cplx d = a.at(col, col);
    for (int j = 0; j < n; ++j) { a.at(col, j) /= d; inv.at(col, j) /= d; }
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      cplx f = a.at(r, col);
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) {
        a.at(r, j) -= f * a.at(col, j);
        inv.at(r, j) -= f * inv.at(col, j);
      }
    }
  }
  return inv;
}

// The shifts S+ and S- with the -mf corner (the quark-mass term of DWF),
// acting on a single-colour 5D spinor v[s][spin].
void shift_plus(const Params &P, const cplx *v, cplx *out) {
  for (int s = 0; s < P.Ls; ++s)
    for (int sp = 0; sp < 4; ++sp)
      out[4 * s + sp] = (s < P.Ls - 1) ? v[4 * (s + 1) + sp] : -P.mf * v[sp];
}
void shift_minus(const Params &P, const cplx *v, cplx *out) {
  for (int s = 0; s < P.Ls; ++s)
    for (int sp = 0; sp < 4; ++sp)
      out[4 * s + sp] = (s > 0) ? v[4 * (s - 1) + sp] : -P.mf * v[4 * (P.Ls - 1) + sp];
}
void spin_mat(const Mat4 m, const cplx *v, cplx *out, int Ls) {
  for (int s = 0; s < Ls; ++s)
    for (int i = 0; i < 4; ++i) {
      cplx acc = 0;
      for (int j = 0; j < 4; ++j) acc += m[i][j] * v[4 * s + j];
      out[4 * s + i] = acc;
    }
}

// P_chi = P- S+ + P+ S-, built column by column from unit vectors.
Op5 build_Pchi(const Params &P) {
  const Gammas &G = gammas();
  int n = 4 * P.Ls;
  Op5 o = op5_zero(n);
  std::vector<cplx> e(n), a(n), b(n), pa(n), pb(n);
  for (int j = 0; j < n; ++j) {
    std::fill(e.begin(), e.end(), 0.0);
    e[j] = 1;
    shift_plus(P, e.data(), a.data());
    shift_minus(P, e.data(), b.data());
    spin_mat(G.Pminus, a.data(), pa.data(), P.Ls);
    spin_mat(G.Pplus, b.data(), pb.data(), P.Ls);
    for (int i = 0; i < n; ++i) o.at(i, j) = pa[i] + pb[i];
  }
  return o;
}

enum { OP_M5 = 0, OP_M5_DAG, OP_M5INV, OP_M5INV_DAG, OP_MPHI, OP_MPHI_DAG, OP_PCHI, OP_COUNT };

struct Ops5 {
  Op5 op[OP_COUNT];
};

// M_phi = b + c P_chi ;  M_5 = (4 - M5) M_phi + 1 - P_chi  (site-diagonal block of D)
Ops5 build_ops5(const Params &P) {
  int n = 4 * P.Ls;
  Ops5 o;
  Op5 one = op5_identity(n);
  Op5 pchi = build_Pchi(P);
  Op5 mphi = op5_lincomb(P.b, one, P.c, pchi);
  Op5 m5 = op5_lincomb(4.0 - P.M5, mphi, 1.0, op5_lincomb(1.0, one, -1.0, pchi));
  o.op[OP_PCHI] = pchi;
  o.op[OP_MPHI] = mphi;
  o.op[OP_MPHI_DAG] = op5_dagger(mphi);
  o.op[OP_M5] = m5;
  o.op[OP_M5_DAG] = op5_dagger(m5);
  o.op[OP_M5INV] = op5_inverse(m5);
  o.op[OP_M5INV_DAG] = op5_dagger(o.op[OP_M5INV]);
  return o;
}

// ---------------------------------------------------------------- field ops
inline size_t idx(const Params &P, int lex, int s, int spin, int col) {
  return (((size_t)lex * P.Ls + s) * 4 + spin) * 3 + col;
}
Field field(const Params &P) { return Field((size_t)P.V * P.Ls * 12, 0.0); }

// out = T in on the sites of the given parity (parity < 0: all sites); other
// sites of out are zeroed.
void apply5(const Params &P, const Op5 &T, Field &out, const Field &in, int parity) {
  Field res = field(P);
  int n = 4 * P.Ls;
  // nonzero entries of each row, so that the sparse operators stay cheap
  std::vector<std::vector<std::pair<int, cplx>>> rows(n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      if (T.at(i, j) != 0.0) rows[i].push_back({j, T.at(i, j)});
#pragma omp parallel for schedule(static)
  for (int x = 0; x < P.V; ++x) {
    if (parity >= 0 && parity_of(P, x) != parity) continue;
    for (int col = 0; col < 3; ++col)
      for (int i = 0; i < n; ++i) {
        cplx acc = 0;
        for (const auto &e : rows[i]) acc += e.second * in[idx(P, x, e.first / 4, e.first % 4, col)];
        res[idx(P, x, i / 4, i % 4, col)] = acc;
      }
  }
  out.swap(res);
}

// Wilson hop with projector sign sg (Sec. 2.2, definition of D^w, read as the
// gauge-covariant form):
//   out(x) = sum_mu [ (1 - sg g_mu) U_mu(x) in(x+mu) + (1 + sg g_mu) U_mu(x-mu)^+ in(x-mu) ]
// sg = +1 gives H, sg = -1 gives its adjoint H^+ (the adjoint of the stencil:
// transposing the site pair swaps which link and projector go with which
// direction).  Only output sites of out_parity are computed (out_parity < 0:
// all); other sites of out are zeroed.
void hop(const Params &P, const cplx *U, Field &out, const Field &in, int out_parity, int sg) {
  const Gammas &G = gammas();
  Field res = field(P);
#pragma omp parallel for schedule(static)
  for (int x = 0; x < P.V; ++x) {
    if (out_parity >= 0 && parity_of(P, x) != out_parity) continue;
    for (int mu = 0; mu < 4; ++mu)
      for (int dir = +1; dir >= -1; dir -= 2) {
        double phase;
        int y = neighbour(P, x, mu, dir, &phase);
        // link: forward U_mu(x), backward U_mu(x-mu)^+
        const cplx *Ufw = U + ((size_t)x * 4 + mu) * 9;
        const cplx *Ubw = U + ((size_t)y * 4 + mu) * 9;
        const Mat4 &proj = (dir > 0) ? (sg > 0 ? G.one_minus[mu] : G.one_plus[mu])
                                     : (sg > 0 ? G.one_plus[mu] : G.one_minus[mu]);
        for (int s = 0; s < P.Ls; ++s) {
          cplx Upsi[4][3];
          for (int sp = 0; sp < 4; ++sp)
            for (int a = 0; a < 3; ++a) {
              cplx acc = 0;
              for (int bb = 0; bb < 3; ++bb) {
                cplx u = (dir > 0) ? Ufw[a * 3 + bb] : std::conj(Ubw[bb * 3 + a]);
                acc += u * in[idx(P, y, s, sp, bb)];
              }
              Upsi[sp][a] = phase * acc;
            }
          for (int sp = 0; sp < 4; ++sp)
            for (int a = 0; a < 3; ++a) {
              cplx acc = 0;
              for (int sq = 0; sq < 4; ++sq) acc += proj[sp][sq] * Upsi[sq][a];
              res[idx(P, x, s, sp, a)] += acc;
            }
        }
      }
  }
  out.swap(res);
}

void axpby(Field &out, cplx a, const Field &x, cplx b, const Field &y) {
  for (size_t i = 0; i < out.size(); ++i) out[i] = a * x[i] + b * y[i];
}
cplx dot(const Field &x, const Field &y) {  // <x,y> = sum conj(x) y
  cplx acc = 0;
  for (size_t i = 0; i < x.size(); ++i) acc += std::conj(x[i]) * y[i];
  return acc;
}
double norm2(const Field &x) {
  double acc = 0;
  for (size_t i = 0; i < x.size(); ++i) acc += std::norm(x[i]);
  return acc;
}
void mask_parity(const Params &P, Field &v, int parity) {
  for (int x = 0; x < P.V; ++x)
    if (parity_of(P, x) != parity)
      for (int k = 0; k < P.Ls * 12; ++k) v[(size_t)x * P.Ls * 12 + k] = 0;
}
// Restrict to the sites of one block (any parity).
void mask_block(const Params &P, const int *nblk, int block, Field &v) {
  for (int x = 0; x < P.V; ++x)
    if (block_of(P, nblk, x) != block)
      for (int k = 0; k < P.Ls * 12; ++k) v[(size_t)x * P.Ls * 12 + k] = 0;
}

// ---------------------------------------------------------------- operators
struct Ctx {
  Params P;
  const cplx *U;
  Ops5 ops;
  // optional truncation (the "sequential Dirichlet" variant of Sec. 2.3):
  // every hop is wrapped as P_s H P_s for block `trunc_block`.
  const int *nblk = nullptr;
  int trunc_block = -1;
};

void hop_ctx(const Ctx &C, Field &out, const Field &in, int out_parity, int sg) {
  if (C.trunc_block < 0) { hop(C.P, C.U, out, in, out_parity, sg); return; }
  Field t = in;
  mask_block(C.P, C.nblk, C.trunc_block, t);
  hop(C.P, C.U, out, t, out_parity, sg);
  mask_block(C.P, C.nblk, C.trunc_block, out);
}

// M^4 from parity 1-p to parity p (Sec. 2.2): M^4 = D^w M_phi with D^w = -H/2.
void M4(const Ctx &C, Field &out, const Field &in, int p) {
  Field t;
  apply5(C.P, C.ops.op[OP_MPHI], t, in, 1 - p);
  hop_ctx(C, out, t, p, +1);
  for (auto &v : out) v *= -0.5;
}
// (M^4_{q, 1-q})^+ : maps parity q to parity p = 1-q;  = -1/2 M_phi^+ H^+.
void M4dag(const Ctx &C, Field &out, const Field &in, int p) {
  Field t;
  hop_ctx(C, t, in, p, -1);
  apply5(C.P, C.ops.op[OP_MPHI_DAG], out, t, p);
  for (auto &v : out) v *= -0.5;
}

// Schur complement on parity p (Sec. 2.2): D_PC = M_5 - M^4_{p,1-p} M_5^{-1} M^4_{1-p,p}
void Dpc(const Ctx &C, Field &out, const Field &in, int p) {
  Field a, b, c, d;
  M4(C, a, in, 1 - p);
  apply5(C.P, C.ops.op[OP_M5INV], b, a, 1 - p);
  M4(C, c, b, p);
  apply5(C.P, C.ops.op[OP_M5], d, in, p);
  out.resize(d.size());
  axpby(out, 1.0, d, -1.0, c);
}
// Its adjoint: D_PC^+ = M_5^+ - (M^4_{1-p,p})^+ M_5^{-+} (M^4_{p,1-p})^+
void Dpc_dag(const Ctx &C, Field &out, const Field &in, int p) {
  Field a, b, c, d;
  M4dag(C, a, in, 1 - p);
  apply5(C.P, C.ops.op[OP_M5INV_DAG], b, a, 1 - p);
  M4dag(C, c, b, p);
  apply5(C.P, C.ops.op[OP_M5_DAG], d, in, p);
  out.resize(d.size());
  axpby(out, 1.0, d, -1.0, c);
}
// Normal operator (Sec. 2.2, normal equation): A = D_PC^+ D_PC
void mdagm(const Ctx &C, Field &out, const Field &in, int p) {
  Field t;
  Dpc(C, t, in, p);
  Dpc_dag(C, out, t, p);
}

// Local operator of block s with snake terms (Sec. 2.3, Sec. 2.4):
//   A_s = P_s A P_s  -- the principal submatrix of the full normal operator.
// With truncated != 0, the sequentially truncated variant (every hop
// replaced by P_s H P_s), which drops the snake terms.
void block_op(const Ctx &C0, const int *nblk, int s, int truncated, Field &out, const Field &in) {
  Ctx C = C0;
  C.nblk = nblk;
  C.trunc_block = truncated ? s : -1;
  Field t = in;
  mask_block(C.P, nblk, s, t);
  mdagm(C, out, t, 0);
  mask_block(C.P, nblk, s, out);
}

// Textbook CG for a fixed number k of iterations from a zero guess
// (Sec. 3: "inner iterations"; Sec. 2.4: zero initial guess, one sweep).
// If the residual or the curvature <p,A p> vanishes the iteration stops and
// keeps the current iterate.  tol > 0: the precision-based stopping that
// Sec. 3 sets aside -- stop after the first iteration whose residual norm is
// at most tol times the initial one (k is then the maximum).
void cg_fixed(const Ctx &C, const int *nblk, int s, int truncated, int k, Field &x, const Field &rhs,
              double tol = 0.0) {
  const Params &P = C.P;
  x = field(P);
  Field r = rhs, p = rhs, q;
  double rr = norm2(r);
  const double rr0 = rr;
  for (int it = 0; it < k; ++it) {
    if (rr == 0.0) break;
    block_op(C, nblk, s, truncated, q, p);
    double pq = std::real(dot(p, q));
    if (pq == 0.0) break;
    double alpha = rr / pq;
    for (size_t i = 0; i < x.size(); ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
    double rr_new = norm2(r);
    if (tol > 0.0 && rr_new <= tol * tol * rr0) break;
    double beta = rr_new / rr;
    for (size_t i = 0; i < p.size(); ++i) p[i] = r[i] + beta * p[i];
    rr = rr_new;
  }
}

// Preconditioner of Sec. 2.4: z = M^{-1} r with M = (+)_s A_s, each block's
// system solved by k inner CG iterations: z = sum_s P_s CG_k(A_s, P_s r).
void local_block_cg(const Ctx &C, const int *nblk, int k, int truncated, Field &z, const Field &r,
                    double tol = 0.0) {
  const Params &P = C.P;
  int nb = nblk[0] * nblk[1] * nblk[2] * nblk[3];
  z = field(P);
  for (int s = 0; s < nb; ++s) {
    Field rs = r, zs;
    mask_block(P, nblk, s, rs);
    mask_parity(P, rs, 0);
    cg_fixed(C, nblk, s, truncated, k, zs, rs, tol);
    for (size_t i = 0; i < z.size(); ++i) z[i] += zs[i];
  }
}

// Multisplitting with several sweeps (Sec. 2.1: the multisplitting
// iteration; Sec. 2.4 keeps one sweep from a zero guess): each further sweep
// solves the blocks again on the residual of the current iterate, so that the
// neighbouring blocks' data enter through A z:  z <- z + M (r - A z).
void multisplit(const Ctx &C, const int *nblk, int k, int truncated, double tol, int sweeps, Field &z,
                const Field &r) {
  local_block_cg(C, nblk, k, truncated, z, r, tol);
  for (int sw = 1; sw < sweeps; ++sw) {
    Field az, t, dz;
    mdagm(C, az, z, 0);
    t.resize(r.size());
    axpby(t, 1.0, r, -1.0, az);
    local_block_cg(C, nblk, k, truncated, dz, t, tol);
    for (size_t i = 0; i < z.size(); ++i) z[i] += dz[i];
  }
}

// Preconditioned CG, Algorithm 1 of Sec. 2.4, on A x = b (even sites).
// Convergence reading: the recursive residual test ||r|| <= tol ||b|| is
// confirmed by the true residual b - A x, which also replaces r every
// `reliable` iterations (reliable update; p is kept).
// nblk == nullptr: M = 1 (plain CG, the comparison of Sec. 3).
// flexible != 0: instead of the printed beta = <z', r'> / <z, r>
// (Fletcher-Reeves), the Polak-Ribiere form beta = <z', r' - r> / <z, r>,
// with r the residual before this iteration's update and r' the one the new
// z' was computed from -- an option for preconditioners that are not fixed
// linear maps (not the paper's algorithm).
struct SolveResult { int iters; double true_rel; int converged; };

SolveResult pcg(const Ctx &C, const int *nblk, int k, int truncated, double tol, int maxiter,
                int reliable, Field &x, const Field &b, double *hist, int hist_len, double inner_tol = 0.0,
                int sweeps = 1, int flexible = 0) {
  const Params &P = C.P;
  auto precond = [&](Field &z, const Field &r) {
    if (nblk) multisplit(C, nblk, k, truncated, inner_tol, sweeps, z, r);
    else z = r;
  };
  double bb = norm2(b);
  SolveResult res{0, 0.0, 0};
  if (bb == 0.0) { x = field(P); res.converged = 1; return res; }
  Field r, q, z, p;
  mdagm(C, q, x, 0);
  r.resize(b.size());
  axpby(r, 1.0, b, -1.0, q);
  double rr = norm2(r);
  if (hist && hist_len > 0) hist[0] = std::sqrt(rr / bb);
  if (rr <= tol * tol * bb) { res.true_rel = std::sqrt(rr / bb); res.converged = 1; return res; }
  precond(z, r);
  p = z;
  double rho = std::real(dot(r, z));
  int it = 0;
  Field r_old;
  while (it < maxiter) {
    mdagm(C, q, p, 0);
    double alpha = rho / std::real(dot(p, q));
    if (flexible) r_old = r;
    for (size_t i = 0; i < x.size(); ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
    ++it;
    rr = norm2(r);
    bool check = rr <= tol * tol * bb;
    if (check || (reliable > 0 && it % reliable == 0)) {
      mdagm(C, q, x, 0);
      axpby(r, 1.0, b, -1.0, q);
      rr = norm2(r);
      if (rr <= tol * tol * bb) { res.converged = 1; }
    }
    if (hist && it < hist_len) hist[it] = std::sqrt(rr / bb);
    if (res.converged) break;
    precond(z, r);
    double rho_new = std::real(dot(z, r));
    double beta = flexible ? (rho_new - std::real(dot(z, r_old))) / rho : rho_new / rho;
    for (size_t i = 0; i < p.size(); ++i) p[i] = z[i] + beta * p[i];
    rho = rho_new;
  }
  res.iters = it;
  mdagm(C, q, x, 0);
  axpby(r, 1.0, b, -1.0, q);
  res.true_rel = std::sqrt(norm2(r) / bb);
  return res;
}

// ---------------------------------------------------------------- packing
// parity-packed [cb][s][spin][col] <-> full lexicographic field
void unpack(const Params &P, Field &full, const double *cbf, int parity) {
  full = field(P);
  const cplx *src = reinterpret_cast<const cplx *>(cbf);
  for (int x = 0; x < P.V; ++x) {
    if (parity_of(P, x) != parity) continue;
    int cb = x >> 1;
    for (int k = 0; k < P.Ls * 12; ++k) full[(size_t)x * P.Ls * 12 + k] = src[(size_t)cb * P.Ls * 12 + k];
  }
}
void pack(const Params &P, double *cbf, const Field &full, int parity) {
  cplx *dst = reinterpret_cast<cplx *>(cbf);
  for (int x = 0; x < P.V; ++x) {
    if (parity_of(P, x) != parity) continue;
    int cb = x >> 1;
    for (int k = 0; k < P.Ls * 12; ++k) dst[(size_t)cb * P.Ls * 12 + k] = full[(size_t)x * P.Ls * 12 + k];
  }
}

bool make_ctx(const int *L, int Ls, const double *p, const double *U, Ctx &C) {
  if (!make_params(L, Ls, p, C.P) || !U) return false;
  C.U = reinterpret_cast<const cplx *>(U);
  C.ops = build_ops5(C.P);
  return true;
}

bool valid_blocks(const Params &P, const int *nblk) {
  if (!nblk) return false;
  for (int mu = 0; mu < 4; ++mu)
    if (nblk[mu] < 1 || nblk[mu] > P.L[mu]) return false;
  return true;
}

}  // namespace

// =====================================================================
// C interface.  Common arguments:
//   L[4]   lattice extents (each even), Ls >= 2 the fifth-dimension extent
//   p[5]   {M5, mf, b, c, tbc}: domain-wall height, quark mass, Moebius b and
//          c (Shamir: b=1, c=0), time boundary factor (-1 antiperiodic)
//   U      gauge field, [lex][mu][row][col][re,im] FP64
//   parity-packed fields as described at the top of this file
// Return 0 on success, -1 on invalid arguments.
// =====================================================================
extern "C" {

int oracle_num_threads(void) { return omp_get_max_threads(); }
void oracle_set_num_threads(int n) { if (n > 0) omp_set_num_threads(n); }

// lex index of each cb site of the parity, and its 8 neighbours' cb indices,
// nbr[cb][mu][0 = forward, 1 = backward].
int oracle_site_maps(const int *L, int parity, int32_t *lex_of_cb, int32_t *nbr) {
  Params P;
  double dummy[5] = {0, 0, 1, 0, -1};
  if (!make_params(L, 2, dummy, P) || (parity & ~1)) return -1;
  for (int x = 0; x < P.V; ++x) {
    if (parity_of(P, x) != parity) continue;
    int cb = x >> 1;
    if (lex_of_cb) lex_of_cb[cb] = x;
    if (nbr)
      for (int mu = 0; mu < 4; ++mu) {
        nbr[(cb * 4 + mu) * 2 + 0] = neighbour(P, x, mu, +1, nullptr) >> 1;
        nbr[(cb * 4 + mu) * 2 + 1] = neighbour(P, x, mu, -1, nullptr) >> 1;
      }
  }
  return 0;
}

int oracle_block_of_site(const int *L, const int *nblk, int32_t *block_of_lex) {
  Params P;
  double dummy[5] = {0, 0, 1, 0, -1};
  if (!make_params(L, 2, dummy, P) || !valid_blocks(P, nblk)) return -1;
  for (int x = 0; x < P.V; ++x) block_of_lex[x] = block_of(P, nblk, x);
  return 0;
}

// The 5D-local matrices as dense (4Ls)^2 complex arrays, index (4s+spin, 4s'+spin').
// which: 0 M_5, 1 M_5^+, 2 M_5^{-1}, 3 M_5^{-+}, 4 M_phi, 5 M_phi^+, 6 P_chi
int oracle_op5_matrix(int Ls, const double *p, int which, double *mat) {
  int L[4] = {2, 2, 2, 2};
  Params P;
  if (!make_params(L, Ls, p, P) || which < 0 || which >= OP_COUNT) return -1;
  Ops5 o = build_ops5(P);
  std::memcpy(mat, o.op[which].m.data(), o.op[which].m.size() * sizeof(cplx));
  return 0;
}

// Full-lattice (lex layout [lex][s][spin][col]) Wilson hop, sg = +1: H, -1: H^+.
int oracle_hop_full(const int *L, int Ls, const double *p, const double *U, double *out,
                    const double *in, int sg) {
  Ctx C;
  if (!make_ctx(L, Ls, p, U, C)) return -1;
  Field f((cplx *)in, (cplx *)in + (size_t)C.P.V * Ls * 12), o;
  hop(C.P, C.U, o, f, -1, sg);
  std::memcpy(out, o.data(), o.size() * sizeof(cplx));
  return 0;
}

// Full 5D Moebius DWF operator D = D_W (b + c P_chi) + (1 - P_chi), D_W = (4-M5) - H/2,
// on lex-layout fields (Sec. 2.2, the operator whose even-odd form is the 2x2 block matrix).
int oracle_D_full(const int *L, int Ls, const double *p, const double *U, double *out, const double *in) {
  Ctx C;
  if (!make_ctx(L, Ls, p, U, C)) return -1;
  const Params &P = C.P;
  Field f((cplx *)in, (cplx *)in + (size_t)P.V * Ls * 12), t, h, pc, o = field(P);
  apply5(P, C.ops.op[OP_MPHI], t, f, -1);
  hop(P, C.U, h, t, -1, +1);
  apply5(P, C.ops.op[OP_PCHI], pc, f, -1);
  for (size_t i = 0; i < o.size(); ++i) o[i] = (4.0 - P.M5) * t[i] - 0.5 * h[i] + f[i] - pc[i];
  std::memcpy(out, o.data(), o.size() * sizeof(cplx));
  return 0;
}

// out (parity p) = M^4_{p,1-p} in (dagger = 0) or (M^4_{1-p,p})^+ in (dagger = 1).
int oracle_dslash_eo(const int *L, int Ls, const double *p, const double *U, double *out,
                     const double *in, int out_parity, int dagger) {
  Ctx C;
  if (!make_ctx(L, Ls, p, U, C) || (out_parity & ~1)) return -1;
  Field f, o;
  unpack(C.P, f, in, 1 - out_parity);
  if (dagger) M4dag(C, o, f, out_parity);
  else M4(C, o, f, out_parity);
  pack(C.P, out, o, out_parity);
  return 0;
}

// out = X in on one parity, X = oracle_op5_matrix(which)
int oracle_op5(const int *L, int Ls, const double *p, double *out, const double *in, int parity, int which) {
  Params P;
  if (!make_params(L, Ls, p, P) || which < 0 || which >= OP_COUNT || (parity & ~1)) return -1;
  Ops5 o = build_ops5(P);
  Field f, r;
  unpack(P, f, in, parity);
  apply5(P, o.op[which], r, f, parity);
  pack(P, out, r, parity);
  return 0;
}

int oracle_dpc(const int *L, int Ls, const double *p, const double *U, double *out, const double *in,
               int parity, int dagger) {
  Ctx C;
  if (!make_ctx(L, Ls, p, U, C) || (parity & ~1)) return -1;
  Field f, o;
  unpack(C.P, f, in, parity);
  if (dagger) Dpc_dag(C, o, f, parity);
  else Dpc(C, o, f, parity);
  pack(C.P, out, o, parity);
  return 0;
}

int oracle_mdagm(const int *L, int Ls, const double *p, const double *U, double *out, const double *in) {
  Ctx C;
  if (!make_ctx(L, Ls, p, U, C)) return -1;
  Field f, o;
  unpack(C.P, f, in, 0);
  mdagm(C, o, f, 0);
  pack(C.P, out, o, 0);
  return 0;
}

// Source preparation (Sec. 2.2): phihat_e = phi_e - M^4_eo M_5^{-1} phi_o and the
// normal-equation right-hand side b = D_PC^+ phihat_e.  phi is lex layout.
int oracle_prepare_rhs(const int *L, int Ls, const double *p, const double *U, double *b_even,
                       double *phihat_even, const double *phi_lex) {
  Ctx C;
  if (!make_ctx(L, Ls, p, U, C)) return -1;
  const Params &P = C.P;
  Field phi((cplx *)phi_lex, (cplx *)phi_lex + (size_t)P.V * Ls * 12);
  Field pe = phi, po = phi, t, u, ph, bb;
  mask_parity(P, pe, 0);
  mask_parity(P, po, 1);
  apply5(P, C.ops.op[OP_M5INV], t, po, 1);
  M4(C, u, t, 0);
  ph.resize(pe.size());
  axpby(ph, 1.0, pe, -1.0, u);
  Dpc_dag(C, bb, ph, 0);
  if (b_even) pack(P, b_even, bb, 0);
  if (phihat_even) pack(P, phihat_even, ph, 0);
  return 0;
}

// Reconstruction: psi_o = M_5^{-1}(phi_o - M^4_oe psi_e); writes the full psi (lex).
int oracle_reconstruct(const int *L, int Ls, const double *p, const double *U, double *psi_lex,
                       const double *psi_even, const double *phi_lex) {
  Ctx C;
  if (!make_ctx(L, Ls, p, U, C)) return -1;
  const Params &P = C.P;
  Field pe, phi((cplx *)phi_lex, (cplx *)phi_lex + (size_t)P.V * Ls * 12), u, t, po;
  unpack(P, pe, psi_even, 0);
  mask_parity(P, phi, 1);
  M4(C, u, pe, 1);
  t.resize(u.size());
  axpby(t, 1.0, phi, -1.0, u);
  apply5(P, C.ops.op[OP_M5INV], po, t, 1);
  for (size_t i = 0; i < po.size(); ++i) po[i] += pe[i];
  std::memcpy(psi_lex, po.data(), po.size() * sizeof(cplx));
  return 0;
}

// out = A_s in on even sites (A_s = P_s A P_s; truncated != 0: no snake terms)
int oracle_block_op(const int *L, int Ls, const double *p, const double *U, double *out,
                    const double *in, const int *nblk, int block, int truncated) {
  Ctx C;
  if (!make_ctx(L, Ls, p, U, C) || !valid_blocks(C.P, nblk)) return -1;
  int nb = nblk[0] * nblk[1] * nblk[2] * nblk[3];
  if (block < 0 || block >= nb) return -1;
  Field f, o;
  unpack(C.P, f, in, 0);
  block_op(C, nblk, block, truncated, o, f);
  pack(C.P, out, o, 0);
  return 0;
}

// z = sum_s P_s CG_k(A_s, P_s r) on even sites
int oracle_local_block_cg(const int *L, int Ls, const double *p, const double *U, double *z,
                          const double *r, const int *nblk, int k, int truncated, double inner_tol, int sweeps) {
  Ctx C;
  if (!make_ctx(L, Ls, p, U, C) || !valid_blocks(C.P, nblk) || k < 0 || !(inner_tol >= 0.0) || sweeps < 0)
    return -1;
  Field rf, zf;
  unpack(C.P, rf, r, 0);
  multisplit(C, nblk, k, truncated, inner_tol, sweeps, zf, rf);
  pack(C.P, z, zf, 0);
  return 0;
}

// Algorithm 1 on the normal equation A x = b (even sites).  x holds the initial
// guess on entry and the solution on exit.  nblk == NULL: plain CG.
// out_stats[0] = outer iterations, [1] = true relative residual ||b-Ax||/||b||,
// [2] = 1 if converged.  hist (optional) receives ||r_k||/||b|| for k < hist_len.
int oracle_solve(const int *L, int Ls, const double *p, const double *U, double *x, const double *b,
                 const int *nblk, int k, int truncated, double tol, int maxiter, int reliable,
                 double *out_stats, double *hist, int hist_len, double inner_tol, int sweeps, int flexible) {
  Ctx C;
  if (!make_ctx(L, Ls, p, U, C) || (nblk && !valid_blocks(C.P, nblk)) || maxiter < 0 || !(inner_tol >= 0.0) ||
      sweeps < 0)
    return -1;
  Field xf, bf;
  unpack(C.P, xf, x, 0);
  unpack(C.P, bf, b, 0);
  SolveResult r = pcg(C, nblk, k, truncated, tol, maxiter, reliable, xf, bf, hist, hist_len, inner_tol, sweeps,
                      flexible);
  pack(C.P, x, xf, 0);
  if (out_stats) { out_stats[0] = r.iters; out_stats[1] = r.true_rel; out_stats[2] = r.converged; }
  return 0;
}

}  // extern "C"
