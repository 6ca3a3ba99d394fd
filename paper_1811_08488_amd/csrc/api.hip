// C-ABI entry points: handle, geometry tables, operators, the batched block
// CG preconditioner and the two FP64 outer solvers (Algorithm 1 with and
// without the multisplitting preconditioner).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

// Scratch of the allocation-free entry point mdagm_noalloc: its two
// intermediate fields (each 256-byte aligned).  One copy per GPU, alive from
// the library's first use on that GPU until the process ends.  Host code
// never names it directly: the device address comes from hipGetSymbolAddress
// (scratch_address below), resolved once per device.
static __device__ __align__(256) unsigned char scratch[MSPCG_NOALLOC_SCRATCH_BYTES];

namespace mspcg {
// Precision-based inner stopping (inner_stop.hip): mode 0 after the initial
// block scalars, 1 after alpha, 2 after the new residual norm.
hipError_t inner_stop(int mode, int nblocks, int nrhs, double tol, double *scal, double *stop, hipStream_t st);
}  // namespace mspcg

using namespace mspcg;

namespace {

thread_local std::string g_last_error;

struct Fail {
  mspcg_status st;
};

void fail(mspcg_status st, const std::string &msg) {
  g_last_error = msg;
  throw Fail{st};
}

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) fail(MSPCG_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Device buffer owned by the handle.
struct DBuf {
  void *p = nullptr;
  size_t bytes = 0;
  DBuf() = default;
  DBuf(const DBuf &) = delete;
  DBuf &operator=(const DBuf &) = delete;
  ~DBuf() {
    if (p) (void)hipFree(p);
  }
  void ensure(size_t n) {
    if (n <= bytes) return;
    if (p) {
      (void)hipFree(p);
      p = nullptr;
      bytes = 0;
    }
    if (n == 0) return;
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      fail(MSPCG_ENOMEM, "device allocation of " + std::to_string(n) + " bytes failed");
    }
    bytes = n;
    // new buffers start at zero (block lists rely on their never-written zero
    // sites).  The clear is ordered on the null stream, which does not order
    // against the solvers' non-blocking stream or a caller's: wait for it
    // before any kernel can touch the buffer (allocation is first-use only,
    // never inside a graph capture).
    HIPCHK(hipMemset(p, 0, n));
    HIPCHK(hipDeviceSynchronize());
  }
  template <typename T> T *as() const { return reinterpret_cast<T *>(p); }
};

template <typename T>
void upload(DBuf &b, const std::vector<T> &v, hipStream_t st) {
  b.ensure(v.size() * sizeof(T) + 16);
  if (!v.empty()) HIPCHK(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
}

size_t prec_bytes(int prec) { return prec == MSPCG_F64 ? 8 : prec == MSPCG_F32 ? 4 : 2; }
bool prec_norm(int prec) { return prec == MSPCG_F16 || prec == MSPCG_BF16; }

// A [nrhs][nsites][Ls][24] vector of one precision owned by the handle.
struct OwnedVec {
  DBuf data, norm;
  Vec v;
  void ensure(int prec, int nrhs, long long nsites, int Ls) {
    const size_t n5 = (size_t)nrhs * nsites * Ls;
    data.ensure(n5 * 24 * prec_bytes(prec));
    if (prec_norm(prec)) norm.ensure(n5 * sizeof(float));
    v.data = data.p;
    v.norm = prec_norm(prec) ? norm.as<float>() : nullptr;
    v.prec = prec;
    v.stride = nsites;
  }
};

// Halo-extended block domains of one blocking (Sec. 2.3: the block operator
// keeps every path of the four hops that leaves the block and comes back).
struct BlockGeom {
  int nblk[4];
  int no_snake = 0;  // 1: every hop cut at the block boundary (O1 = odd, E2 = even sites of the block)
  int nb = 0;
  int be_tot = 0, o1_tot = 0, e2_tot = 0;
  std::vector<int> be_off, o1_off, e2_off;   // padded offsets, size nb+1
  std::vector<int> be_n, o1_n, e2_n;         // true counts
  std::vector<int> be_lex, o1_lex, e2_lex;   // lex per padded entry (-1 padding)
  DBuf d_be_cb, d_be_blk, d_be_nbr, d_be_e2, d_o1_cb, d_o1_nbr_be, d_o1_nbr_e2, d_e2_cb, d_e2_nbr, d_e2_be, d_be_off,
      d_e2_off;
  // work vectors (inner precision); `gen` changes whenever they are reallocated
  // or cleared for another layout, so that graphs captured on them are never replayed
  int vprec = -1, vnrhs = 0;
  long long gen = 0;
  OwnedVec x, r, p, mp, Ap, o1v, e2v;  // mp = M_phi p, the first hop's input
  DBuf stopbuf;  // precision-based inner stopping: [nb * nrhs][2] (inner_stop.hip)
  DBuf partial, scal, rrbuf;
};

constexpr int kPad = 64;  // zero sites after a block list; block lists are padded to multiples of block_align

// Block lists are padded to a multiple of this many sites, so that workgroups
// of the block kernels (any power of two up to 64 sites) and the whole-wave
// site counts of the hop layout (G sites of one right-hand side fill a wave)
// never straddle two blocks: 64, or 64 G when G is not a power of two.
int block_align(int Ls) {
  const int G = hop_groups_per_wave(Ls, 1);  // the layout of one right-hand side (a multiple for the others)
  return (G > 0 && (G & (G - 1)) != 0) ? kPad * G : kPad;
}

// The chain coefficients of a fifth-dimension operator in FP64 and FP32 (the
// compute types of the kernels).
struct Mat5 {
  DBuf d, f;
  const void *ptr(int prec) const { return prec == MSPCG_F64 ? d.p : f.p; }
};

}  // namespace

namespace {
// Device address of `scratch` on the current device, looked up once per device.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices] = {};

void *scratch_address() {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) fail(MSPCG_EUNSUPPORTED, "device ordinal above the scratch table size");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void *ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) fail(MSPCG_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_addr[dev] = ptr;
  }
  return g_scratch_addr[dev];
}
}  // namespace

struct mspcg_handle {
  mspcg_dwf par;
  int device = -1;                    // the HIP device the handle was created on
  void *scratch_dev = nullptr;        // that device's copy of `scratch` (mdagm_noalloc)
  int V = 0, Vh = 0, Lxyz = 0;
  hipStream_t stream = nullptr;       // caller's stream given at creation (set-up work)
  hipStream_t work = nullptr;         // the solvers' own stream (default priority, capturable)
  // captured preconditioner launches, keyed by everything they bake in
  std::map<std::vector<intptr_t>, hipGraphExec_t> graphs;
  double alpha5 = 0, beta5 = 0;  // M_5 = alpha5 - beta5 P_chi
  // global tables per parity: site list (identity), neighbours (cb of the other parity)
  DBuf d_order[2], d_nbr[2], d_lex[2], d_nbrlex[2];
  std::vector<int> lex_of_cb[2], nbr_cb[2];
  DBuf links[4][2];
  bool links_ok[4] = {false, false, false, false};
  DBuf d_gauge;
  // fifth-dimension operators as chain coefficients (kChainHead + Ls values, F64 and F32 copies)
  Mat5 m5inv, x1;  // chain coefficients of M_5^{-1} and of M_phi M_5^{-1} (the kernels also apply the transposes)
  // FP64 workspaces
  OwnedVec tmp_o, tmp_e, tmp_o2, tmp_e2, sr, sp, sq, sz;
  OwnedVec sw_t, sw_z, sw_q;  // multisplitting sweeps: r - A z, the sweep's correction, A z
  OwnedVec lbc_r, lbc_z;      // local_block_cg on F32 fields: F64 copies of r and z
  DBuf partial, scal;
  std::map<std::vector<int>, std::unique_ptr<BlockGeom>> blocks;
  // sites per workgroup chosen by the autotuner, per kernel variant and shape
  std::map<std::vector<int>, int> tuned;
  bool autotune = true;
  int verbose = 0;  // MSPCG_VERBOSE=n: the solvers report progress on stderr every n outer iterations
  ~mspcg_handle() {
    if (work) (void)hipStreamSynchronize(work);
    for (auto &g : graphs) (void)hipGraphExecDestroy(g.second);
    if (work) (void)hipStreamDestroy(work);
  }
};

namespace {

template <typename F>
mspcg_status guarded(F &&f) {
  try {
    g_last_error.clear();
    f();
    return MSPCG_OK;
  } catch (const Fail &e) {
    return e.st;
  } catch (const std::exception &e) {
    g_last_error = e.what();
    return MSPCG_EINVAL;
  } catch (...) {
    g_last_error = "unknown error";
    return MSPCG_EINVAL;
  }
}

hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

// sites per workgroup: the largest power of two with <= 256 threads (>= 1)
int pick_nsite(int nrhs, int Ls) {
  int n = 1;
  while (n * 2 <= kPad && hop_threads(Ls, nrhs, n * 2) <= 256) n *= 2;
  return n;
}

// ------------------------------------------------------------- fifth dimension
// Chain coefficients (see kChainHead) of X = (b_phi / alpha)(1 + rho S)(1 - q S)^{-1},
// q = beta / alpha, per chirality: M_5^{-1} with rho = 0, b_phi = 1 and
// M_phi M_5^{-1} = (b + c S)(alpha - beta S)^{-1} with rho = c / b, b_phi = b
// (S^Ls = -mf, so (1 - q S)^{-1} = sum_k q^k S^k / (1 + mf q^Ls)).
std::vector<double> chain_coefs(int Ls, double alpha, double beta, double mf, double rho, double b_phi) {
  const double q = beta / alpha;
  const double gamma = -q * mf / (1.0 + mf * std::pow(q, Ls));
  std::vector<double> c(kChainHead + Ls);
  c[0] = rho;
  c[1] = -rho * mf;
  c[2] = q;
  c[3] = b_phi / alpha;
  double qi = 1.0;
  for (int i = 0; i < Ls; ++i, qi *= q) c[kChainHead + i] = gamma * qi;
  return c;
}

// ------------------------------------------------------------- validation
void check_field(mspcg_handle *h, const mspcg_field *f, const char *name) {
  if (!f || !f->data) fail(MSPCG_EINVAL, std::string(name) + ": NULL field");
  if (f->nrhs < 1) fail(MSPCG_EINVAL, std::string(name) + ": nrhs < 1");
  if (f->nrhs > MSPCG_MAX_NRHS) fail(MSPCG_EUNSUPPORTED, std::string(name) + ": nrhs above MSPCG_MAX_NRHS");
  if (f->parity != 0 && f->parity != 1) fail(MSPCG_EINVAL, std::string(name) + ": parity must be 0 or 1");
  if (f->prec < MSPCG_F64 || f->prec > MSPCG_BF16) fail(MSPCG_EINVAL, std::string(name) + ": unknown precision");
  if (prec_norm(f->prec) && !f->norm) fail(MSPCG_EINVAL, std::string(name) + ": F16/BF16 field without norm array");
  if (hop_threads(h->par.Ls, f->nrhs, 1) > 256)
    fail(MSPCG_EUNSUPPORTED, std::string(name) + ": one site's nrhs x Ls lanes exceed a 256-thread workgroup");
}

Vec vec_of(mspcg_handle *h, const mspcg_field *f) {
  Vec v;
  v.data = f->data;
  v.norm = f->norm;
  v.prec = f->prec;
  v.stride = h->Vh;
  return v;
}

// ------------------------------------------------------------- gauge / links
void ensure_links(mspcg_handle *h, int prec, hipStream_t st) {
  if (h->links_ok[prec]) return;
  for (int p = 0; p < 2; ++p) {
    h->links[prec][p].ensure((size_t)h->Vh * 8 * 18 * prec_bytes(prec));
    HIPCHK(pack_links(prec, h->links[prec][p].p, h->d_gauge.as<double>(), h->d_lex[p].as<int>(),
                      h->d_nbrlex[p].as<int>(), p, h->Vh, h->par.L[3], h->Lxyz, (double)h->par.t_bc, st));
  }
  h->links_ok[prec] = true;
}

// ------------------------------------------------------------- hop launches
HopArgs base_args(mspcg_handle *h, int nrhs) {
  HopArgs a;
  std::memset(&a, 0, sizeof(a));
  a.Ls = h->par.Ls;
  a.nrhs = nrhs;
  a.nsite_wg = pick_nsite(nrhs, h->par.Ls);
  a.mphi_b = h->par.b;
  a.mphi_c = h->par.c;
  a.mf = h->par.mf;
  a.m5_alpha = h->alpha5;
  a.m5_beta = h->beta5;
  return a;
}

// Launch a hop with the tuned number of sites per workgroup; returns the grid
// size (= number of partial sums written when `dot`).  The first launch of a
// variant/shape times every candidate with HIP events on the stream (the
// kernels are pure functions of their inputs, so repeating them is harmless)
// and keeps the fastest; the default shape wins ties within 3%.
// may_tune = false (the allocation-free entry points): no timing, no events;
// an untuned shape launches with the default and stays untuned.
// the autotuner's key: kernel variant, list and shape
std::vector<int> hop_key(int list_kind, int prec, int dag, int pre, int epi, int dot, int global, const HopArgs &a) {
  return {list_kind, prec, dag, pre, epi, dot, global, a.Ls, a.nrhs, a.nsites};
}

int run_hop(mspcg_handle *h, int list_kind, int prec, int dag, int pre, int epi, int dot, int global, HopArgs a,
            hipStream_t st, bool may_tune = true) {
  const std::vector<int> key = hop_key(list_kind, prec, dag, pre, epi, dot, global, a);
  auto it = h->tuned.find(key);
  int n = 0;
  if (it != h->tuned.end()) {
    n = it->second;
  } else {
    // Candidates: powers of two up to kPad, and the site counts that fill
    // whole waves when Ls does not divide 64 (multiples of 5 sites for
    // Ls = 12).  A block-list hop with a fused dot product reduces per block,
    // so its workgroups must not straddle blocks: only divisors of the block
    // alignment.
    const int G = hop_groups_per_wave(a.Ls, a.nrhs);
    const int al = block_align(a.Ls);
    auto allowed = [&](int c) { return global || !dot || al % c == 0; };
    std::vector<int> cands;
    for (int c = 1; c <= kPad; c *= 2) cands.push_back(c);
    if (G > 0)
      for (int w = 1; w <= 4; ++w)
        if ((G * w) % a.nrhs == 0 && allowed(G * w / a.nrhs) &&
            std::find(cands.begin(), cands.end(), G * w / a.nrhs) == cands.end())
          cands.push_back(G * w / a.nrhs);
    int n0 = pick_nsite(a.nrhs, a.Ls);
    if (G > 0)  // default: the fullest workgroup of whole waves
      for (int w = 4; w >= 1; --w)
        if ((G * w) % a.nrhs == 0 && allowed(G * w / a.nrhs) && hop_threads(a.Ls, a.nrhs, G * w / a.nrhs) <= 256) {
          n0 = G * w / a.nrhs;
          break;
        }
    n = n0;
    if (h->autotune && may_tune) {
      hipEvent_t e0, e1;
      HIPCHK(hipEventCreate(&e0));
      HIPCHK(hipEventCreate(&e1));
      float best = 0;
      for (int c : cands) {
        const int thr = hop_threads(a.Ls, a.nrhs, c);
        if (thr > 256 || (thr < 64 && hop_threads(a.Ls, a.nrhs, 2 * c) <= 256 && c < kPad)) continue;
        a.nsite_wg = c;
        if (launch_hop(prec, dag, pre, epi, dot, global, a, st) != hipSuccess) {
          (void)hipGetLastError();
          continue;
        }
        HIPCHK(hipEventRecord(e0, st));
        for (int rep = 0; rep < 3; ++rep) HIPCHK(launch_hop(prec, dag, pre, epi, dot, global, a, st));
        HIPCHK(hipEventRecord(e1, st));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        if (c == n0) ms *= 0.97f;
        if (best == 0 || ms < best) {
          best = ms;
          n = c;
        }
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
    }
    if (may_tune) h->tuned[key] = n;
  }
  a.nsite_wg = n;
  HIPCHK(launch_hop(prec, dag, pre, epi, dot, global, a, st));
  return (a.nsites + n - 1) / n;
}

// Full-lattice hop: output parity p (site list = all cb), input parity 1-p.
int global_hop(mspcg_handle *h, int prec, int nrhs, int p, const Vec &out, const Vec &in, int dag, int pre, int epi,
               double scale, const Mat5 *mat, const Vec *other, double *partial, const Vec *dotw,
               hipStream_t st, bool may_tune = true) {
  if (may_tune) ensure_links(h, prec, st);
  else if (!h->links_ok[prec]) fail(MSPCG_EUNSUPPORTED, "links of this precision have not been prepared");
  HopArgs a = base_args(h, nrhs);
  a.nsites = h->Vh;
  a.site_cb = h->d_order[p].as<int>();
  a.nbr = h->d_nbr[p].as<int>();
  a.in = in.data;
  a.in_norm = in.norm;
  a.in_stride = h->Vh;
  a.out = out.data;
  a.out_norm = out.norm;
  a.out_stride = h->Vh;
  a.links = h->links[prec][p].p;
  a.scale = scale;
  a.mat = mat ? mat->ptr(prec) : nullptr;
  if (other) {
    a.other = other->data;
    a.other_norm = other->norm;
    a.other_stride = h->Vh;
  }
  if (partial) {
    a.partial = partial;
    a.dotw = dotw->data;
    a.dotw_norm = dotw->norm;
    a.dotw_stride = h->Vh;
  }
  return run_hop(h, 0, prec, dag, pre, epi, partial ? 1 : 0, 1, a, st, may_tune);
}

// out_e = D_PC^+ D_PC in_e (all four hops fused with their fifth-dimension
// neighbours); optional partial Re<in, out> per workgroup.
int apply_mdagm(mspcg_handle *h, int prec, int nrhs, const Vec &out, const Vec &in, const Vec &to, const Vec &te,
                double *partial, hipStream_t st, bool may_tune = true) {
  // c_o = M_phi M_5^{-1} (-1/2 H_oe M_phi in)
  global_hop(h, prec, nrhs, 1, to, in, 0, 1, EPI_M5INV, -0.5, &h->x1, nullptr, nullptr, nullptr, st, may_tune);
  // y_e = M_5 in + 1/2 H_eo c_o  (= D_PC in)
  global_hop(h, prec, nrhs, 0, te, to, 0, 0, EPI_M5_OTHER, 0.5, nullptr, &in, nullptr, nullptr, st, may_tune);
  // f_o = M_5^{-+} M_phi^+ (-1/2 H^+_oe y_e)
  global_hop(h, prec, nrhs, 1, to, te, 1, 0, EPI_M5INV, -0.5, &h->x1, nullptr, nullptr, nullptr, st, may_tune);
  // out = M_5^+ y + 1/2 M_phi^+ H^+_eo f  (= D_PC^+ y)
  return global_hop(h, prec, nrhs, 0, out, to, 1, 0, EPI_M5DAG_MPHIDAG, 0.5, nullptr, &te, partial, &in, st,
                    may_tune);
}

void ensure_fp64_temps(mspcg_handle *h, int nrhs) {
  h->tmp_o.ensure(MSPCG_F64, nrhs, h->Vh, h->par.Ls);
  h->tmp_e.ensure(MSPCG_F64, nrhs, h->Vh, h->par.Ls);
}

// ------------------------------------------------------------- block geometry
// no_snake = 0: the domains of A_s = P_s A P_s with its snake terms (halo of
// depth 2); no_snake = 1: the block alone, every hop cut at its boundary
// (P_s H P_s), which drops the snake terms.
BlockGeom *get_blocks(mspcg_handle *h, const int nblk[4], int no_snake, hipStream_t st) {
  std::vector<int> key(nblk, nblk + 4);
  key.push_back(no_snake ? 1 : 0);
  auto it = h->blocks.find(key);
  if (it != h->blocks.end()) return it->second.get();
  const int *L = h->par.L;
  const int depth = no_snake ? 0 : 2;  // halo of the extended domains
  for (int mu = 0; mu < 4; ++mu) {
    if (nblk[mu] < 1 || nblk[mu] > L[mu]) fail(MSPCG_EINVAL, "nblk out of range");
    if (nblk[mu] >= 2 && L[mu] / nblk[mu] + (L[mu] % nblk[mu] ? 1 : 0) + 2 * depth > L[mu])
      fail(MSPCG_EUNSUPPORTED, "block halo of depth 2 would wrap onto itself (need L >= block + 4)");
  }
  auto bg = std::make_unique<BlockGeom>();
  std::memcpy(bg->nblk, nblk, sizeof(bg->nblk));
  bg->no_snake = no_snake ? 1 : 0;
  bg->nb = nblk[0] * nblk[1] * nblk[2] * nblk[3];
  const int V = h->V;
  std::vector<int> e2_of_lex(V, -1), o1_of_lex(V, -1);  // per-block scratch maps
  std::vector<int> be_cb, be_blk, be_nbr, be_e2, o1_cb, o1_nbr_be, o1_nbr_e2, e2_cb, e2_nbr, e2_be;
  bg->be_off.push_back(0);
  bg->o1_off.push_back(0);
  bg->e2_off.push_back(0);
  auto lex_of = [&](const int c[4]) { return c[0] + L[0] * (c[1] + L[1] * (c[2] + L[2] * c[3])); };
  for (int b = 0; b < bg->nb; ++b) {
    int jb[4], start[4], size[4], lo[4], hi[4];
    for (int mu = 0, t = b; mu < 4; ++mu) {
      jb[mu] = t % nblk[mu];
      t /= nblk[mu];
      const int q = L[mu] / nblk[mu], rr = L[mu] % nblk[mu];
      start[mu] = jb[mu] * q + std::min(jb[mu], rr);
      size[mu] = q + (jb[mu] < rr ? 1 : 0);
      lo[mu] = nblk[mu] >= 2 ? -depth : 0;
      hi[mu] = nblk[mu] >= 2 ? size[mu] + depth : size[mu];
    }
    // enumerate the extended box in local lex order (x fastest)
    std::vector<int> loc_be, loc_o1, loc_e2;
    std::vector<int> dist_e2;
    for (int ut = lo[3]; ut < hi[3]; ++ut)
      for (int uz = lo[2]; uz < hi[2]; ++uz)
        for (int uy = lo[1]; uy < hi[1]; ++uy)
          for (int ux = lo[0]; ux < hi[0]; ++ux) {
            const int u[4] = {ux, uy, uz, ut};
            int dist = 0, c[4];
            for (int mu = 0; mu < 4; ++mu) {
              dist += std::max(0, std::max(-u[mu], u[mu] - (size[mu] - 1)));
              c[mu] = ((start[mu] + u[mu]) % L[mu] + L[mu]) % L[mu];
            }
            const int g = lex_of(c);
            const int par = (c[0] + c[1] + c[2] + c[3]) & 1;
            if (par == 0 && dist <= depth) {
              loc_e2.push_back(g);
              dist_e2.push_back(dist);
            }
            if (par == 1 && dist <= depth / 2) loc_o1.push_back(g);
            if (par == 0 && dist == 0) loc_be.push_back(g);
          }
    const int be0 = bg->be_off.back(), o10 = bg->o1_off.back(), e20 = bg->e2_off.back();
    const int nbe = (int)loc_be.size(), no1 = (int)loc_o1.size(), ne2 = (int)loc_e2.size();
    const int al = block_align(h->par.Ls);
    const int pbe = (nbe + al - 1) / al * al, po1 = (no1 + al - 1) / al * al, pe2 = (ne2 + al - 1) / al * al;
    for (int i = 0; i < no1; ++i) o1_of_lex[loc_o1[i]] = o10 + i;
    for (int i = 0; i < ne2; ++i) e2_of_lex[loc_e2[i]] = e20 + i;
    std::vector<int> be_of_e2(ne2, -1);
    {
      int k = 0;
      for (int i = 0; i < ne2; ++i)
        if (dist_e2[i] == 0) be_of_e2[i] = be0 + k++;
    }
    auto nb_lex = [&](int g, int d) {
      int c[4];
      int t = g;
      for (int mu = 0; mu < 4; ++mu) { c[mu] = t % L[mu]; t /= L[mu]; }
      const int mu = d >> 1;
      c[mu] = (c[mu] + ((d & 1) ? -1 : 1) + L[mu]) % L[mu];
      return lex_of(c);
    };
    // E2 (even) -> O1 neighbours, map to B_e
    for (int i = 0; i < pe2; ++i) {
      if (i < ne2) {
        const int g = loc_e2[i];
        e2_cb.push_back(g >> 1);
        for (int d = 0; d < 8; ++d) e2_nbr.push_back(o1_of_lex[nb_lex(g, d)]);
        e2_be.push_back(be_of_e2[i]);
        bg->e2_lex.push_back(g);
      } else {
        e2_cb.push_back(-1);
        for (int d = 0; d < 8; ++d) e2_nbr.push_back(-1);
        e2_be.push_back(-1);
        bg->e2_lex.push_back(-1);
      }
    }
    // O1 (odd) -> E2 / B_e neighbours
    for (int i = 0; i < po1; ++i) {
      if (i < no1) {
        const int g = loc_o1[i];
        o1_cb.push_back(g >> 1);
        for (int d = 0; d < 8; ++d) {
          const int e = e2_of_lex[nb_lex(g, d)];
          o1_nbr_e2.push_back(e);
          o1_nbr_be.push_back(e >= 0 ? be_of_e2[e - e20] : -1);
        }
        bg->o1_lex.push_back(g);
      } else {
        o1_cb.push_back(-1);
        for (int d = 0; d < 8; ++d) { o1_nbr_e2.push_back(-1); o1_nbr_be.push_back(-1); }
        bg->o1_lex.push_back(-1);
      }
    }
    // B_e in block-local lex order; neighbours from its E2 entry
    {
      int k = 0;
      for (int i = 0; i < ne2; ++i) {
        if (dist_e2[i] != 0) continue;
        const int g = loc_e2[i];
        if (g != loc_be[k]) fail(MSPCG_EINVAL, "internal: block ordering mismatch");
        be_cb.push_back(g >> 1);
        be_blk.push_back(b);
        be_e2.push_back(e20 + i);
        for (int d = 0; d < 8; ++d) be_nbr.push_back(e2_nbr[(size_t)(e20 + i) * 8 + d]);
        bg->be_lex.push_back(g);
        ++k;
      }
      for (int i = nbe; i < pbe; ++i) {
        be_cb.push_back(-1);
        be_blk.push_back(-1);
        be_e2.push_back(-1);
        for (int d = 0; d < 8; ++d) be_nbr.push_back(-1);
        bg->be_lex.push_back(-1);
      }
    }
    for (int i = 0; i < no1; ++i) o1_of_lex[loc_o1[i]] = -1;
    for (int i = 0; i < ne2; ++i) e2_of_lex[loc_e2[i]] = -1;
    bg->be_n.push_back(nbe);
    bg->o1_n.push_back(no1);
    bg->e2_n.push_back(ne2);
    bg->be_off.push_back(be0 + pbe);
    bg->o1_off.push_back(o10 + po1);
    bg->e2_off.push_back(e20 + pe2);
  }
  bg->be_tot = bg->be_off.back();
  bg->o1_tot = bg->o1_off.back();
  bg->e2_tot = bg->e2_off.back();
  // Neighbour tables: a neighbour outside the domain (a third of the first
  // hop's, for example) is stored as -1 - alt, alt being an inside neighbour of
  // the same site (or, for a padding site, one of the target list's kPad
  // all-zero extra sites): the kernel loads alt's data, already at hand for
  // another direction, and gives it weight zero, so these reads neither leave
  // the cache nor converge on one all-zero site.
  auto encode_out = [](std::vector<int> &t, int zero) {
    for (size_t row = 0; row * 8 < t.size(); ++row) {
      int alt = -1;
      for (int d = 0; d < 8 && alt < 0; ++d) alt = t[row * 8 + d];
      if (alt < 0) alt = zero + (int)(row % kPad);
      for (int d = 0; d < 8; ++d) {
        int &x = t[row * 8 + d];
        if (x >= zero) fail(MSPCG_EINVAL, "internal: block table out of range");
        if (x < 0) x = -1 - alt;
      }
    }
  };
  encode_out(be_nbr, bg->o1_tot);
  encode_out(e2_nbr, bg->o1_tot);
  encode_out(o1_nbr_e2, bg->e2_tot);
  encode_out(o1_nbr_be, bg->be_tot);
  // `other` index tables: -1 for a site whose operand lies outside (zero, not loaded)
  for (int x : e2_be)
    if (x >= bg->be_tot) fail(MSPCG_EINVAL, "internal: block table out of range");
  for (int x : be_e2)
    if (x >= bg->e2_tot) fail(MSPCG_EINVAL, "internal: block table out of range");
  upload(bg->d_be_cb, be_cb, st);
  upload(bg->d_be_blk, be_blk, st);
  upload(bg->d_be_nbr, be_nbr, st);
  upload(bg->d_be_e2, be_e2, st);
  upload(bg->d_o1_cb, o1_cb, st);
  upload(bg->d_o1_nbr_be, o1_nbr_be, st);
  upload(bg->d_o1_nbr_e2, o1_nbr_e2, st);
  upload(bg->d_e2_cb, e2_cb, st);
  upload(bg->d_e2_nbr, e2_nbr, st);
  upload(bg->d_e2_be, e2_be, st);
  upload(bg->d_be_off, bg->be_off, st);
  upload(bg->d_e2_off, bg->e2_off, st);
  HIPCHK(hipStreamSynchronize(st));
  BlockGeom *raw = bg.get();
  h->blocks[key] = std::move(bg);
  return raw;
}

// Captured preconditioner graphs bake in the block work buffers: drop every
// graph of `bg` (called when they are reallocated or cleared for a relayout;
// the solvers synchronise before returning, so none is in flight).
void drop_block_graphs(mspcg_handle *h, BlockGeom *bg) {
  for (auto it = h->graphs.begin(); it != h->graphs.end();) {
    if (!it->first.empty() && it->first[0] == (intptr_t)bg) {
      (void)hipGraphExecDestroy(it->second);
      it = h->graphs.erase(it);
    } else {
      ++it;
    }
  }
}

void ensure_block_vecs(mspcg_handle *h, BlockGeom *bg, int prec, int nrhs) {
  const int Ls = h->par.Ls;
  const bool relayout = bg->vprec != prec || bg->vnrhs != nrhs;
  const std::vector<void *> before = {bg->x.data.p, bg->x.norm.p, bg->r.data.p, bg->r.norm.p, bg->p.data.p,
                                      bg->p.norm.p, bg->mp.data.p, bg->mp.norm.p, bg->Ap.data.p, bg->Ap.norm.p, bg->o1v.data.p, bg->o1v.norm.p,
                                      bg->e2v.data.p, bg->e2v.norm.p, bg->partial.p, bg->scal.p, bg->rrbuf.p,
                                      bg->stopbuf.p};
  // each list carries kPad extra sites after its last block: never written, so zero
  bg->x.ensure(prec, nrhs, bg->be_tot + kPad, Ls);
  bg->r.ensure(prec, nrhs, bg->be_tot + kPad, Ls);
  bg->p.ensure(prec, nrhs, bg->be_tot + kPad, Ls);
  bg->mp.ensure(prec, nrhs, bg->be_tot + kPad, Ls);
  bg->Ap.ensure(prec, nrhs, bg->be_tot + kPad, Ls);
  bg->o1v.ensure(prec, nrhs, bg->o1_tot + kPad, Ls);
  bg->e2v.ensure(prec, nrhs, bg->e2_tot + kPad, Ls);
  // upper bound on the workgroups of a hop with fused partials (nsite_wg >= 1;
  // the tuner tries 1): the second hop runs on E2, the last on B_e
  const int nwg = std::max(bg->be_tot, bg->e2_tot);
  bg->partial.ensure((size_t)nwg * nrhs * sizeof(double));
  bg->scal.ensure((size_t)bg->nb * nrhs * kScal * sizeof(double));
  bg->rrbuf.ensure((size_t)nrhs * sizeof(double) + 16);
  bg->stopbuf.ensure((size_t)bg->nb * nrhs * 2 * sizeof(double));
  if (relayout) {
    // the zero sites sit at other byte offsets in another precision or nrhs:
    // clear the buffers once so that they hold zeros again
    for (OwnedVec *v : {&bg->x, &bg->r, &bg->p, &bg->mp, &bg->Ap, &bg->o1v, &bg->e2v}) {
      if (v->data.p) HIPCHK(hipMemset(v->data.p, 0, v->data.bytes));
      if (v->norm.p) HIPCHK(hipMemset(v->norm.p, 0, v->norm.bytes));
    }
    HIPCHK(hipDeviceSynchronize());  // as in DBuf::ensure: the null stream orders nothing else
  }
  const std::vector<void *> after = {bg->x.data.p, bg->x.norm.p, bg->r.data.p, bg->r.norm.p, bg->p.data.p,
                                     bg->p.norm.p, bg->mp.data.p, bg->mp.norm.p, bg->Ap.data.p, bg->Ap.norm.p, bg->o1v.data.p, bg->o1v.norm.p,
                                     bg->e2v.data.p, bg->e2v.norm.p, bg->partial.p, bg->scal.p, bg->rrbuf.p,
                                     bg->stopbuf.p};
  if (relayout || before != after) {
    drop_block_graphs(h, bg);
    ++bg->gen;
  }
  bg->vprec = prec;
  bg->vnrhs = nrhs;
}

// Block-domain hop arguments (lists, tables and fields of one hop of A_s).
HopArgs block_hop_args(mspcg_handle *h, int nrhs, int nsites, const int *site_cb, const int *nbr, const Vec &in,
                       const Vec &out, int out_parity, int prec) {
  HopArgs a = base_args(h, nrhs);
  a.nsites = nsites;
  a.site_cb = site_cb;
  a.nbr = nbr;
  a.in = in.data;
  a.in_norm = in.norm;
  a.in_stride = in.stride;
  a.out = out.data;
  a.out_norm = out.norm;
  a.out_stride = out.stride;
  a.links = h->links[prec][out_parity].p;
  return a;
}

// One of the four hops of A_s on the halo-extended domains, for every block at
// once: 1: B_e -> O1, 2: O1 -> E2, 3: E2 -> O1, 4: O1 -> B_e (optional partial
// Re<in, out> per workgroup).  in_mp = M_phi in (formed by the kernels that
// write the block vector).  Returns the grid size of the launch.
// upd_scal (last hop only): instead of storing A_s in, update the block
// residual in place, r <- r - alpha A_s in (alpha from upd_scal per block and
// rhs), with the partials |r|^2 of the stored values.
int block_hop(mspcg_handle *h, BlockGeom *bg, int prec, int nrhs, int which, const Vec &in, const Vec &in_mp,
              const Vec &out, double *partial, hipStream_t st, const double *upd_scal = nullptr) {
  if (which == 1) {  // c = M_phi M_5^{-1} (-1/2 H M_phi in) on O1
    HopArgs a1 = block_hop_args(h, nrhs, bg->o1_tot, bg->d_o1_cb.as<int>(), bg->d_o1_nbr_be.as<int>(), in_mp,
                                bg->o1v.v, 1, prec);
    a1.scale = -0.5;
    a1.mat = h->x1.ptr(prec);
    return run_hop(h, 1, prec, 0, 0, EPI_M5INV, 0, 0, a1, st);
  }
  if (which == 2) {  // y = M_5 in + 1/2 H c on E2
    HopArgs a2 = block_hop_args(h, nrhs, bg->e2_tot, bg->d_e2_cb.as<int>(), bg->d_e2_nbr.as<int>(), bg->o1v.v,
                                bg->e2v.v, 0, prec);
    a2.scale = 0.5;
    a2.other = in.data;
    a2.other_norm = in.norm;
    a2.other_stride = in.stride;
    a2.other_idx = bg->d_e2_be.as<int>();
    // (with partial: |y|^2 per workgroup; y = D_PC P_s in on all of E2, so the
    // sum over a block is <in, A_s in>)
    a2.partial = partial;
    return run_hop(h, 2, prec, 0, 0, EPI_M5_OTHER, partial ? 1 : 0, 0, a2, st);
  }
  if (which == 3) {  // f = M_5^{-+} M_phi^+ (-1/2 H^+ y) on O1
    HopArgs a3 = block_hop_args(h, nrhs, bg->o1_tot, bg->d_o1_cb.as<int>(), bg->d_o1_nbr_e2.as<int>(), bg->e2v.v,
                                bg->o1v.v, 1, prec);
    a3.scale = -0.5;
    a3.mat = h->x1.ptr(prec);  // (the daggered hop applies the transpose)
    return run_hop(h, 3, prec, 1, 0, EPI_M5INV, 0, 0, a3, st);
  }
  // out = M_5^+ y + 1/2 M_phi^+ H^+ f on B_e
  HopArgs a4 = block_hop_args(h, nrhs, bg->be_tot, bg->d_be_cb.as<int>(), bg->d_be_nbr.as<int>(), bg->o1v.v, out,
                              0, prec);
  a4.scale = 0.5;
  a4.other = bg->e2v.v.data;
  a4.other_norm = bg->e2v.v.norm;
  a4.other_stride = bg->e2v.v.stride;
  a4.other_idx = bg->d_be_e2.as<int>();
  if (upd_scal) {
    // The update writes r in place, so the launch must not be repeated: the
    // shape is tuned once on the same kernel writing A_s in into `out`
    // (a scratch vector here), and the updating launch then uses it.
    HopArgs t = a4;
    t.partial = partial;
    if (h->tuned.find(hop_key(4, prec, 1, 0, EPI_M5DAG_MPHIDAG, 1, 0, t)) == h->tuned.end())
      (void)run_hop(h, 4, prec, 1, 0, EPI_M5DAG_MPHIDAG, 1, 0, t, st);
    a4.out = bg->r.v.data;
    a4.out_norm = bg->r.v.norm;
    a4.out_stride = bg->r.v.stride;
    a4.upd_scal = upd_scal;
    a4.upd_blk = bg->d_be_blk.as<int>();
    a4.partial = partial;
    return run_hop(h, 4, prec, 1, 0, EPI_M5DAG_MPHIDAG, 1, 0, a4, st, false);
  }
  if (partial) {
    a4.partial = partial;
    a4.dotw = in.data;
    a4.dotw_norm = in.norm;
    a4.dotw_stride = in.stride;
  }
  return run_hop(h, 4, prec, 1, 0, EPI_M5DAG_MPHIDAG, partial ? 1 : 0, 0, a4, st);
}

// out = A_s in for every block at once on the halo-extended domains
// (B_e -> O1 -> E2 -> O1 -> B_e); optional partial sums of Re<in, out> per
// workgroup.  With the snake terms A_s = P_s D_PC^+ D_PC P_s, so
// <in, A_s in> = |D_PC P_s in|^2 is summed by the second hop over E2 (the
// whole support of D_PC P_s in) from values it already holds, and the last
// hop does not read `in` again; the truncated operator sums Re<in, out> in the
// last hop.  Returns the sites per workgroup of the hop that formed the
// partials and sets *off to that hop's per-block offsets in its list.
int block_hops(mspcg_handle *h, BlockGeom *bg, int prec, int nrhs, const Vec &in, const Vec &in_mp, const Vec &out,
               double *partial, hipStream_t st, const int **off = nullptr) {
  const bool on_e2 = partial && !bg->no_snake;
  block_hop(h, bg, prec, nrhs, 1, in, in_mp, out, nullptr, st);
  const int grid2 = block_hop(h, bg, prec, nrhs, 2, in, in_mp, out, on_e2 ? partial : nullptr, st);
  block_hop(h, bg, prec, nrhs, 3, in, in_mp, out, nullptr, st);
  const int grid4 = block_hop(h, bg, prec, nrhs, 4, in, in_mp, out, on_e2 ? nullptr : partial, st);
  if (off) *off = on_e2 ? bg->d_e2_off.as<int>() : bg->d_be_off.as<int>();
  return on_e2 ? (bg->e2_tot + grid2 - 1) / grid2 : (bg->be_tot + grid4 - 1) / grid4;
}

BlockArgs block_args(mspcg_handle *h, BlockGeom *bg, int nrhs) {
  BlockArgs ba;
  ba.nsites = bg->be_tot;
  ba.Ls = h->par.Ls;
  ba.nrhs = nrhs;
  ba.nsite_wg = pick_nsite(nrhs, h->par.Ls);
  ba.be_cb = bg->d_be_cb.as<int>();
  ba.be_blk = bg->d_be_blk.as<int>();
  ba.nblocks = bg->nb;
  ba.be_off = bg->d_be_off.as<int>();
  ba.mphi_b = h->par.b;
  ba.mphi_c = h->par.c;
  ba.mf = h->par.mf;
  return ba;
}

// What the block state holds after run_block_cg, for the kernels that form z
// from it: 0 = the final iterate in x; 1 = x and the last step alpha p (fixed
// k > 1); 2 = only the step (k = 1).
int scatter_mode(int k, double inner_tol) { return (inner_tol > 0.0 || k < 1) ? 0 : (k == 1 ? 2 : 1); }

// The preconditioner: z = sum_s P_s CG_k(A_s, P_s r) for every (block, rhs).
// r, z: FP64 even fields (z without data: only the partials are formed, and
// block_scatter_xpay takes z from the block state).  rr: device |r|^2 per rhs
// (RMS scaling); partial_zr (optional): workgroup partials of Re<z, r> for the
// outer solver.
void run_block_cg(mspcg_handle *h, BlockGeom *bg, int prec, int nrhs, int k, double inner_tol, const Vec &z,
                  const Vec &r, const double *rr, double *partial_zr, int *nparts_zr, hipStream_t st) {
  ensure_links(h, prec, st);
  ensure_block_vecs(h, bg, prec, nrhs);
  const int Ls = h->par.Ls;
  BlockArgs ba = block_args(h, bg, nrhs);
  const double n_total = (double)h->Vh * Ls * 24;
  double *part = bg->partial.as<double>();
  double *scal = bg->scal.as<double>();
  // inner_tol > 0: precision-based stopping (inner_stop.hip), else exactly k iterations
  const bool stop = inner_tol > 0.0;
  double *stopd = stop ? bg->stopbuf.as<double>() : nullptr;
  // Fixed k >= 1: x_0 = 0 is never stored (the first update sets x = alpha p)
  // and the last iteration's x update happens in the scatter (x + alpha p,
  // with no r update: nothing reads r after it).  Precision-based stopping
  // keeps every step, since its test reads |r|^2 after the last update.
  const int smode = scatter_mode(k, inner_tol);
  const bool lazy_x = smode != 0;
  HIPCHK(block_gather(prec, ba, lazy_x ? Vec() : bg->x.v, bg->r.v, bg->p.v, bg->mp.v, r, rr, n_total, part, st));
  HIPCHK(block_scalars(2, ba, part, scal, st));
  if (lazy_x && !bg->no_snake) {
    // With the snake terms <p, A_s p> = |D_PC P_s p|^2 comes from the second
    // hop, so alpha is known before the third: the last hop updates r in place
    // (no A_s p vector, no separate r pass), and the last iteration, whose
    // A_s p would only update r, stops after the second hop.
    for (int it = 0; it < k; ++it) {
      block_hop(h, bg, prec, nrhs, 1, bg->p.v, bg->mp.v, bg->Ap.v, nullptr, st);
      BlockArgs ba2 = ba;
      const int g2 = block_hop(h, bg, prec, nrhs, 2, bg->p.v, bg->mp.v, bg->Ap.v, part, st);
      ba2.nsite_wg = (bg->e2_tot + g2 - 1) / g2;
      ba2.be_off = bg->d_e2_off.as<int>();
      HIPCHK(block_scalars(0, ba2, part, scal, st));
      if (it + 1 == k) break;
      block_hop(h, bg, prec, nrhs, 3, bg->p.v, bg->mp.v, bg->Ap.v, nullptr, st);
      BlockArgs ba4 = ba;
      const int g4 = block_hop(h, bg, prec, nrhs, 4, bg->p.v, bg->mp.v, bg->Ap.v, part, st, scal);
      ba4.nsite_wg = (bg->be_tot + g4 - 1) / g4;
      HIPCHK(block_scalars(1, ba4, part, scal, st));
      HIPCHK(block_update_xp(prec, ba, bg->x.v, bg->p.v, bg->mp.v, bg->r.v, scal, it == 0, st));
    }
    HIPCHK(block_scatter(prec, ba, z, bg->x.v, bg->p.v, scal, smode, r, rr, n_total, partial_zr ? partial_zr : part,
                         st));
    if (nparts_zr) *nparts_zr = (ba.nsites + ba.nsite_wg - 1) / ba.nsite_wg;
    return;
  }
  if (stop) HIPCHK(inner_stop(0, bg->nb, nrhs, inner_tol, scal, stopd, st));
  for (int it = 0; it < k; ++it) {
    BlockArgs ba4 = ba;
    ba4.nsite_wg = block_hops(h, bg, prec, nrhs, bg->p.v, bg->mp.v, bg->Ap.v, part, st, &ba4.be_off);
    HIPCHK(block_scalars(0, ba4, part, scal, st));
    if (stop) HIPCHK(inner_stop(1, bg->nb, nrhs, inner_tol, scal, stopd, st));
    if (it + 1 < k) {
      // r first (its norm gives beta), then x and p in one pass
      HIPCHK(block_update_r(prec, ba, bg->r.v, bg->Ap.v, scal, part, st));
      HIPCHK(block_scalars(1, ba, part, scal, st));
      if (stop) HIPCHK(inner_stop(2, bg->nb, nrhs, inner_tol, scal, stopd, st));
      HIPCHK(block_update_xp(prec, ba, bg->x.v, bg->p.v, bg->mp.v, bg->r.v, scal, lazy_x && it == 0, st));
    } else if (!lazy_x) {
      HIPCHK(block_update_xr(prec, ba, bg->x.v, bg->r.v, bg->p.v, bg->Ap.v, scal, part, st));
    }
  }
  HIPCHK(block_scatter(prec, ba, z, bg->x.v, bg->p.v, scal, smode, r, rr, n_total, partial_zr ? partial_zr : part,
                       st));
  if (nparts_zr) *nparts_zr = (ba.nsites + ba.nsite_wg - 1) / ba.nsite_wg;
}

// Further multisplitting sweeps (Sec. 2.1) after the first one in z:
// z <- z + M (r - A z), M the one-sweep preconditioner applied by `apply_M`
// (z, r, |r|^2 per rhs); FP64 temporaries owned by the handle.
template <typename ApplyM>
void more_sweeps(mspcg_handle *h, int nrhs, int sweeps, const Vec &z, const Vec &r, double *rr_tmp, double *part,
                 hipStream_t st, ApplyM apply_M) {
  const int Ls = h->par.Ls;
  const long long n = (long long)h->Vh * Ls * 24;
  h->sw_t.ensure(MSPCG_F64, nrhs, h->Vh, Ls);
  h->sw_z.ensure(MSPCG_F64, nrhs, h->Vh, Ls);
  h->sw_q.ensure(MSPCG_F64, nrhs, h->Vh, Ls);
  ensure_fp64_temps(h, nrhs);
  double *zd = (double *)z.data, *rd = (double *)r.data;
  double *td = (double *)h->sw_t.v.data, *z2 = (double *)h->sw_z.v.data, *qd = (double *)h->sw_q.v.data;
  for (int sw = 1; sw < sweeps; ++sw) {
    apply_mdagm(h, MSPCG_F64, nrhs, h->sw_q.v, z, h->tmp_o.v, h->tmp_e.v, nullptr, st);
    HIPCHK(blas_axpby(td, 1.0, rd, -1.0, qd, n, nrhs, st));  // t = r - A z
    HIPCHK(blas_dot_partial(td, td, n, nrhs, part, st));
    HIPCHK(blas_reduce(part, kBlasGrid, nrhs, rr_tmp, st));
    apply_M(h->sw_z.v, h->sw_t.v, rr_tmp);
    HIPCHK(blas_axpby(zd, 1.0, zd, 1.0, z2, n, nrhs, st));  // z += M t
  }
}

// ------------------------------------------------------------- solvers
struct SolverWork {
  double *rho, *pap, *alpha, *beta, *rr, *bb, *tmp, *rrt, *zrt, *zq;
  int *active;
};

// Time split of a solve: an event is recorded on the solver's stream at each
// phase boundary, tagged with the phase that starts there; the time of a phase
// is the elapsed time to the next event.  Completed intervals are summed at
// the solver's host synchronisations and their events recycled.
struct PhaseTimer {
  enum { OP = 0, PRECOND = 1, BLAS = 2 };
  bool on = false;
  hipStream_t st = nullptr;
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<hipEvent_t, int>> marks;
  double t[3] = {0, 0, 0};
  void mark(int phase) {
    if (!on) return;
    hipEvent_t e;
    if (pool.empty()) {
      HIPCHK(hipEventCreate(&e));
    } else {
      e = pool.back();
      pool.pop_back();
    }
    HIPCHK(hipEventRecord(e, st));
    marks.emplace_back(e, phase);
  }
  // after a synchronisation of the stream: every interval but the open last one is complete
  void drain() {
    if (!on || marks.size() < 2) return;
    for (size_t i = 0; i + 1 < marks.size(); ++i) {
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, marks[i].first, marks[i + 1].first));
      t[marks[i].second] += 1e-3 * ms;
      pool.push_back(marks[i].first);
    }
    marks.erase(marks.begin(), marks.end() - 1);
  }
  ~PhaseTimer() {
    for (auto &m : marks) (void)hipEventDestroy(m.first);
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

mspcg_status solve(mspcg_handle *h, mspcg_field *x, const mspcg_field *b, const mspcg_solver *s,
                   const mspcg_precond *pc, mspcg_stats *st_out) {
  mspcg_status result = MSPCG_OK;
  mspcg_status rc = guarded([&] {
    const auto t0 = std::chrono::steady_clock::now();
    if (!h || !s) fail(MSPCG_EINVAL, "NULL handle or solver parameters");
    check_field(h, x, "x");
    check_field(h, b, "b");
    if (x->prec != MSPCG_F64 || b->prec != MSPCG_F64) fail(MSPCG_EINVAL, "solvers take F64 fields");
    if (x->parity != 0 || b->parity != 0) fail(MSPCG_EINVAL, "solvers work on even sites");
    if (x->nrhs != b->nrhs) fail(MSPCG_EINVAL, "x and b differ in nrhs");
    if (!(s->tol > 0) || s->max_iter < 0 || s->reliable_interval < 0) fail(MSPCG_EINVAL, "bad solver parameters");
    if (pc) {
      if (pc->n_inner < 0) fail(MSPCG_EINVAL, "n_inner < 0");
      if (pc->inner_prec < MSPCG_F64 || pc->inner_prec > MSPCG_BF16) fail(MSPCG_EINVAL, "bad inner precision");
      if (!(pc->inner_tol >= 0.0) || !std::isfinite(pc->inner_tol)) fail(MSPCG_EINVAL, "inner_tol < 0 or not finite");
      if (pc->n_sweeps < 0) fail(MSPCG_EINVAL, "n_sweeps < 0");
    }
    // the caller's fields may still be written by work on other streams
    HIPCHK(hipDeviceSynchronize());
    hipStream_t st = h->work;
    const int nrhs = b->nrhs, Ls = h->par.Ls;
    const long long n = (long long)h->Vh * Ls * 24;
    BlockGeom *bg = pc ? get_blocks(h, pc->nblk, pc->no_snake, st) : nullptr;
    ensure_fp64_temps(h, nrhs);
    h->sr.ensure(MSPCG_F64, nrhs, h->Vh, Ls);
    h->sp.ensure(MSPCG_F64, nrhs, h->Vh, Ls);
    h->sq.ensure(MSPCG_F64, nrhs, h->Vh, Ls);
    if (pc) h->sz.ensure(MSPCG_F64, nrhs, h->Vh, Ls);
    const size_t nparts_max = std::max<size_t>((size_t)std::max(h->Vh, kBlasGrid), bg ? (size_t)bg->be_tot : 0);
    h->partial.ensure(nparts_max * nrhs * sizeof(double));
    h->scal.ensure((size_t)nrhs * 11 * sizeof(double) + 64);
    double *part = h->partial.as<double>();
    SolverWork w;
    w.rho = h->scal.as<double>();
    w.pap = w.rho + nrhs;
    w.alpha = w.pap + nrhs;
    w.beta = w.alpha + nrhs;
    w.rr = w.beta + nrhs;
    w.bb = w.rr + nrhs;
    w.tmp = w.bb + nrhs;
    w.rrt = w.tmp + nrhs;
    w.zrt = w.rrt + nrhs;
    w.zq = w.zrt + nrhs;
    w.active = reinterpret_cast<int *>(w.zq + nrhs);
    PhaseTimer tm;
    tm.on = s->timing != 0;
    tm.st = st;
    tm.mark(PhaseTimer::BLAS);
    Vec X = vec_of(h, x), B = vec_of(h, b), R = h->sr.v, P = h->sp.v, Q = h->sq.v;
    Vec Z = pc ? h->sz.v : R;
    double *xd = (double *)X.data, *bd = (double *)B.data, *rd = (double *)R.data, *pd = (double *)P.data,
           *qd = (double *)Q.data, *zd = (double *)Z.data;
    std::vector<double> hb(nrhs), hr(nrhs);
    std::vector<int> active(nrhs, 1);
    auto norm2 = [&](const double *v, double *out) {
      HIPCHK(blas_dot_partial(v, v, n, nrhs, part, st));
      HIPCHK(blas_reduce(part, kBlasGrid, nrhs, out, st));
    };
    auto to_host = [&](const double *d, std::vector<double> &hv) {
      HIPCHK(hipMemcpyAsync(hv.data(), d, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      tm.drain();
      for (double v : hv)
        if (!std::isfinite(v)) fail(MSPCG_ENONFINITE, "non-finite value in a solver reduction");
    };
    auto push_active = [&] {
      HIPCHK(hipMemcpyAsync(w.active, active.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, st));
    };
    auto true_residual = [&] {  // r = b - A x, rr
      tm.mark(PhaseTimer::OP);
      apply_mdagm(h, MSPCG_F64, nrhs, Q, X, h->tmp_o.v, h->tmp_e.v, nullptr, st);
      tm.mark(PhaseTimer::BLAS);
      HIPCHK(blas_axpby(rd, 1.0, bd, -1.0, qd, n, nrhs, st));
      norm2(rd, w.rr);
      to_host(w.rr, hr);
    };
    // one sweep of the preconditioner: zv = M rv with <zv, rv> into zrv (rrv: |rv|^2)
    auto precond_one = [&](const Vec &Zv, const Vec &Rv, double *rrv, double *zrv) {
      auto precond_launch = [&] {
        int nparts = 0;
        run_block_cg(h, bg, pc->inner_prec, nrhs, pc->n_inner, pc->inner_tol, Zv, Rv, rrv, part, &nparts, st);
        HIPCHK(blas_reduce(part, nparts, nrhs, zrv, st));
      };
      if (!s->use_graph) {
        precond_launch();
        return;
      }
      // size (and, for another precision or nrhs, clear) the block buffers before
      // the key is formed: the key names their generation
      ensure_links(h, pc->inner_prec, st);
      ensure_block_vecs(h, bg, pc->inner_prec, nrhs);
      int64_t tol_bits;
      std::memcpy(&tol_bits, &pc->inner_tol, sizeof tol_bits);
      const std::vector<intptr_t> key = {(intptr_t)bg, (intptr_t)bg->gen, pc->inner_prec, nrhs, pc->n_inner,
                                         (intptr_t)tol_bits, (intptr_t)Zv.data, (intptr_t)Rv.data, (intptr_t)rrv,
                                         (intptr_t)part, (intptr_t)zrv};
      auto it = h->graphs.find(key);
      if (it != h->graphs.end()) {
        HIPCHK(hipGraphLaunch(it->second, st));
        return;
      }
      // first use: run eagerly (tunes launch shapes and sizes every buffer), then
      // capture the identical launch sequence for the following iterations
      precond_launch();
      hipGraph_t graph = nullptr;
      HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      try {
        precond_launch();
      } catch (...) {
        (void)hipStreamEndCapture(st, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        throw;
      }
      HIPCHK(hipStreamEndCapture(st, &graph));
      hipGraphExec_t exec = nullptr;
      const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      HIPCHK(e);
      h->graphs[key] = exec;
    };
    // One sweep with the Fletcher-Reeves beta: z is never stored; the direction
    // update p = z + beta p reads it from the block state (block_scatter_xpay)
    const bool fuse_p = pc && !s->flexible_beta && pc->n_sweeps <= 1;
    auto update_p = [&](bool first) {  // p = z (first) or z + beta p
      if (fuse_p) {
        tm.mark(PhaseTimer::PRECOND);
        HIPCHK(block_scatter_xpay(pc->inner_prec, block_args(h, bg, nrhs), P, bg->x.v, bg->p.v,
                                  bg->scal.as<double>(), scatter_mode(pc->n_inner, pc->inner_tol), w.rr,
                                  (double)h->Vh * Ls * 24, w.beta, first ? 1 : 0, st));
        tm.mark(PhaseTimer::BLAS);
      } else if (first) {
        HIPCHK(blas_axpby(pd, 1.0, zd, 0.0, zd, n, nrhs, st));
      } else {
        HIPCHK(blas_xpay(pd, zd, w.beta, n, nrhs, st));
      }
    };
    auto precond = [&] {  // z = M^{-1} r and rho_new = <z, r> into w.tmp
      if (!pc) {
        HIPCHK(hipMemcpyAsync(w.tmp, w.rr, nrhs * sizeof(double), hipMemcpyDeviceToDevice, st));
        return;
      }
      tm.mark(PhaseTimer::PRECOND);
      precond_one(fuse_p ? Vec() : Z, R, w.rr, w.tmp);
      if (pc->n_sweeps > 1) {
        more_sweeps(h, nrhs, pc->n_sweeps, Z, R, w.rrt, part, st,
                    [&](const Vec &z2, const Vec &t, double *rrt) { precond_one(z2, t, rrt, w.zrt); });
        HIPCHK(blas_dot_partial(zd, rd, n, nrhs, part, st));
        HIPCHK(blas_reduce(part, kBlasGrid, nrhs, w.tmp, st));
      }
      tm.mark(PhaseTimer::BLAS);
    };
    const double tol2 = s->tol * s->tol;
    norm2(bd, w.bb);
    to_host(w.bb, hb);
    for (int i = 0; i < nrhs; ++i)
      if (hb[i] == 0.0) active[i] = 0;
    // b = 0: x = 0 is the solution
    for (int i = 0; i < nrhs; ++i)
      if (hb[i] == 0.0) HIPCHK(hipMemsetAsync(xd + (size_t)i * n, 0, n * sizeof(double), st));
    true_residual();
    for (int i = 0; i < nrhs; ++i)
      if (active[i] && hr[i] <= tol2 * hb[i]) active[i] = 0;
    push_active();
    int it = 0;
    long long inner = 0;
    bool any = false;
    for (int a : active) any |= (a != 0);
    if (any) {
      precond();
      if (pc) inner += (long long)pc->n_inner * std::max(1, pc->n_sweeps);
      update_p(true);  // p = z
      HIPCHK(hipMemcpyAsync(w.rho, w.tmp, nrhs * sizeof(double), hipMemcpyDeviceToDevice, st));
      while (it < s->max_iter) {
        tm.mark(PhaseTimer::OP);
        const int hop_parts = apply_mdagm(h, MSPCG_F64, nrhs, Q, P, h->tmp_o.v, h->tmp_e.v, part, st);
        tm.mark(PhaseTimer::BLAS);
        HIPCHK(blas_reduce(part, hop_parts, nrhs, w.pap, st));
        HIPCHK(solver_scalars(0, nrhs, w.active, w.rho, w.pap, w.alpha, st));
        HIPCHK(blas_update_xr(xd, rd, pd, qd, w.alpha, n, nrhs, part, st));
        HIPCHK(blas_reduce(part, kBlasGrid, nrhs, w.rr, st));
        ++it;
        to_host(w.rr, hr);
        bool check = false;
        for (int i = 0; i < nrhs; ++i) check |= active[i] && hr[i] <= tol2 * hb[i];
        const bool reliable = s->reliable_interval > 0 && it % s->reliable_interval == 0;
        if (check || reliable) {
          true_residual();
          bool changed = false;
          for (int i = 0; i < nrhs; ++i)
            if (active[i] && hr[i] <= tol2 * hb[i]) { active[i] = 0; changed = true; }
          if (changed) push_active();
        }
        if (h->verbose > 0 && it % h->verbose == 0) {
          double worst = 0;
          for (int i = 0; i < nrhs; ++i)
            if (hb[i] > 0) worst = std::max(worst, std::sqrt(hr[i] / hb[i]));
          std::fprintf(stderr, "[mspcg] %s iteration %d: relative residual %.3e, %.1f s\n", pc ? "MSPCG" : "CG", it,
                       worst, std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
        }
        any = false;
        for (int a : active) any |= (a != 0);
        if (!any) break;
        precond();
        if (pc) inner += (long long)pc->n_inner * std::max(1, pc->n_sweeps);
        if (s->flexible_beta) {
          // Polak-Ribiere: beta = <z', r' - r> / <z, r> with r' - r = -alpha A p
          // (q still holds A p), i.e. beta = -<z', A p> / <p, A p>
          HIPCHK(blas_dot_partial(zd, qd, n, nrhs, part, st));
          HIPCHK(blas_reduce(part, kBlasGrid, nrhs, w.zq, st));
          HIPCHK(solver_scalars(2, nrhs, w.active, w.rho, w.tmp, w.beta, st, w.zq, w.pap));
        } else {
          HIPCHK(solver_scalars(1, nrhs, w.active, w.rho, w.tmp, w.beta, st));
        }
        update_p(false);
      }
    }
    // final true residual
    true_residual();
    tm.mark(PhaseTimer::BLAS);
    bool conv = true;
    for (int i = 0; i < nrhs; ++i) {
      const double rel = hb[i] > 0 ? std::sqrt(hr[i] / hb[i]) : 0.0;
      if (hb[i] > 0 && !(rel <= s->tol)) conv = false;
      if (st_out && st_out->true_rel_resid) st_out->true_rel_resid[i] = rel;
    }
    HIPCHK(hipStreamSynchronize(st));
    tm.drain();
    if (st_out) {
      st_out->outer_iters = it;
      st_out->inner_iters = inner;
      st_out->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      st_out->t_outer_op = tm.t[PhaseTimer::OP];
      st_out->t_precond = tm.t[PhaseTimer::PRECOND];
      st_out->t_blas = tm.t[PhaseTimer::BLAS];
    }
    result = conv ? MSPCG_OK : MSPCG_NOT_CONVERGED;
  });
  return rc != MSPCG_OK ? rc : result;
}

}  // namespace

// =================================================================== C ABI
extern "C" {

const char *mspcg_last_error(void) { return g_last_error.c_str(); }

mspcg_status mspcg_create(mspcg_handle **hp, const mspcg_dwf *p, const double *gauge, void *stream) {
  if (!hp) {
    g_last_error = "NULL handle pointer";
    return MSPCG_EINVAL;
  }
  *hp = nullptr;
  std::unique_ptr<mspcg_handle> h(new mspcg_handle);
  mspcg_status rc = guarded([&] {
    if (!p || !gauge) fail(MSPCG_EINVAL, "NULL parameters or gauge field");
    for (int mu = 0; mu < 4; ++mu)
      if (p->L[mu] < 2 || (p->L[mu] & 1)) fail(MSPCG_EINVAL, "every lattice extent must be even and >= 2");
    if (p->Ls < 2) fail(MSPCG_EINVAL, "Ls < 2");
    if (p->Ls > MSPCG_MAX_LS) fail(MSPCG_EUNSUPPORTED, "Ls above MSPCG_MAX_LS");
    if (p->t_bc != 1 && p->t_bc != -1) fail(MSPCG_EINVAL, "t_bc must be +1 or -1");
    if (!std::isfinite(p->M5) || !std::isfinite(p->mf) || !std::isfinite(p->b) || !std::isfinite(p->c))
      fail(MSPCG_EINVAL, "non-finite action parameter");
    long long V = 1;
    for (int mu = 0; mu < 4; ++mu) V *= p->L[mu];
    if (V > (1LL << 30)) fail(MSPCG_EUNSUPPORTED, "lattice volume too large for 32-bit site indices");
    h->par = *p;
    h->V = (int)V;
    h->Vh = (int)(V / 2);
    h->Lxyz = p->L[0] * p->L[1] * p->L[2];
    h->stream = S(stream);
    HIPCHK(hipGetDevice(&h->device));
    h->scratch_dev = scratch_address();
    HIPCHK(hipStreamCreateWithFlags(&h->work, hipStreamNonBlocking));
    if (const char *e = std::getenv("MSPCG_AUTOTUNE")) h->autotune = std::atoi(e) != 0;
    if (const char *e = std::getenv("MSPCG_VERBOSE")) h->verbose = std::max(0, std::atoi(e));
    h->alpha5 = p->b * (4.0 - p->M5) + 1.0;
    h->beta5 = 1.0 - p->c * (4.0 - p->M5);
    const int Ls = p->Ls;
    const double q = h->beta5 / h->alpha5;
    if (std::abs(1 + p->mf * std::pow(q, Ls)) < 1e-300 || h->alpha5 == 0.0) fail(MSPCG_EINVAL, "M_5 is singular");
    if (p->b == 0.0) fail(MSPCG_EUNSUPPORTED, "Moebius b = 0 is not supported");
    hipStream_t st = h->stream;
    // index maps
    const int *L = p->L;
    const int Lxh = L[0] / 2;
    // output sites of the full-lattice hop are visited column by column: the
    // lattice is cut into columns of 12x12x12 spatial sites (8 where 12 does
    // not divide an extent, the full extent where neither does) running the
    // whole time direction, and each column is swept along t.  Consecutive workgroups (one XCD each range, see the
    // kernels' workgroup renumbering) then need only a few neighbouring time
    // slices of one column at a time, which stay in that XCD's L2.
    int cdim[3];
    for (int mu = 0; mu < 3; ++mu) cdim[mu] = (L[mu] % 12 == 0) ? 12 : (L[mu] % 8 == 0) ? 8 : L[mu];
    if (const char *e = std::getenv("MSPCG_SITE_TILE")) {  // "x,y,z": spatial extent of the sweep's columns
      int t[3];
      if (std::sscanf(e, "%d,%d,%d", &t[0], &t[1], &t[2]) == 3 && t[0] > 0 && t[1] > 0 && t[2] > 0 &&
          L[0] % t[0] == 0 && L[1] % t[1] == 0 && L[2] % t[2] == 0)
        for (int mu = 0; mu < 3; ++mu) cdim[mu] = t[mu];
    }
    for (int par = 0; par < 2; ++par) {
      std::vector<int> order;
      order.reserve(h->Vh);
      for (int bz = 0; bz < L[2]; bz += cdim[2])
        for (int by = 0; by < L[1]; by += cdim[1])
          for (int bx = 0; bx < L[0]; bx += cdim[0])
            for (int t = 0; t < L[3]; ++t)
              for (int z = bz; z < bz + cdim[2]; ++z)
                for (int y = by; y < by + cdim[1]; ++y)
                  for (int x = bx; x < bx + cdim[0]; ++x)
                    if (((x + y + z + t) & 1) == par) order.push_back((x + L[0] * (y + L[1] * (z + L[2] * t))) >> 1);
      if ((int)order.size() != h->Vh) fail(MSPCG_EINVAL, "internal: site order incomplete");
      upload(h->d_order[par], order, st);
    }
    for (int par = 0; par < 2; ++par) {
      auto &lex = h->lex_of_cb[par];
      auto &nbr = h->nbr_cb[par];
      std::vector<int> nbrlex((size_t)h->Vh * 8);
      lex.resize(h->Vh);
      nbr.resize((size_t)h->Vh * 8);
      for (int cb = 0; cb < h->Vh; ++cb) {
        int c[4];
        int rest = cb / Lxh;
        c[1] = rest % L[1];
        c[2] = (rest / L[1]) % L[2];
        c[3] = rest / (L[1] * L[2]);
        c[0] = 2 * (cb % Lxh) + ((par + c[1] + c[2] + c[3]) & 1);
        lex[cb] = c[0] + L[0] * (c[1] + L[1] * (c[2] + L[2] * c[3]));
        for (int d = 0; d < 8; ++d) {
          int y[4] = {c[0], c[1], c[2], c[3]};
          const int mu = d >> 1;
          y[mu] = (y[mu] + ((d & 1) ? -1 : 1) + L[mu]) % L[mu];
          const int yl = y[0] + L[0] * (y[1] + L[1] * (y[2] + L[2] * y[3]));
          nbrlex[(size_t)cb * 8 + d] = yl;
          nbr[(size_t)cb * 8 + d] = yl >> 1;
        }
      }
      upload(h->d_lex[par], lex, st);
      upload(h->d_nbr[par], nbr, st);
      upload(h->d_nbrlex[par], nbrlex, st);
    }
    // gauge copy (physical links) for repacking in any precision
    h->d_gauge.ensure((size_t)V * 4 * 18 * sizeof(double));
    HIPCHK(hipMemcpyAsync(h->d_gauge.p, gauge, (size_t)V * 4 * 18 * sizeof(double), hipMemcpyDeviceToDevice, st));
    ensure_links(h.get(), MSPCG_F64, st);
    // fifth-dimension operators as chain coefficients
    auto up5 = [&](Mat5 &m, const std::vector<double> &v) {
      upload(m.d, v, st);
      upload(m.f, std::vector<float>(v.begin(), v.end()), st);
    };
    up5(h->m5inv, chain_coefs(Ls, h->alpha5, h->beta5, p->mf, 0.0, 1.0));
    up5(h->x1, chain_coefs(Ls, h->alpha5, h->beta5, p->mf, p->c / p->b, p->b));
    HIPCHK(hipStreamSynchronize(st));
  });
  if (rc == MSPCG_OK) *hp = h.release();
  return rc;
}

mspcg_status mspcg_destroy(mspcg_handle *h) {
  if (!h) return MSPCG_OK;
  (void)hipStreamSynchronize(h->stream);
  delete h;
  return MSPCG_OK;
}

mspcg_status dslash_eo(mspcg_handle *h, mspcg_field *out, const mspcg_field *in, int dagger, void *stream) {
  return guarded([&] {
    if (!h) fail(MSPCG_EINVAL, "NULL handle");
    check_field(h, out, "out");
    check_field(h, in, "in");
    if (out->parity == in->parity) fail(MSPCG_EINVAL, "dslash_eo: out and in must have opposite parity");
    if (out->prec != in->prec || out->nrhs != in->nrhs) fail(MSPCG_EINVAL, "dslash_eo: precision/nrhs mismatch");
    if (out->data == in->data) fail(MSPCG_EINVAL, "dslash_eo: out must not alias in");
    const Vec o = vec_of(h, out), i = vec_of(h, in);
    if (!dagger)
      global_hop(h, in->prec, in->nrhs, out->parity, o, i, 0, 1, EPI_SCALE, -0.5, nullptr, nullptr, nullptr, nullptr,
                 S(stream));
    else
      global_hop(h, in->prec, in->nrhs, out->parity, o, i, 1, 0, EPI_MPHIDAG, -0.5, nullptr, nullptr, nullptr, nullptr,
                 S(stream));
  });
}

mspcg_status m5inv(mspcg_handle *h, mspcg_field *out, const mspcg_field *in, int dagger, void *stream) {
  return guarded([&] {
    if (!h) fail(MSPCG_EINVAL, "NULL handle");
    check_field(h, out, "out");
    check_field(h, in, "in");
    if (out->parity != in->parity) fail(MSPCG_EINVAL, "m5inv: out and in must have the same parity");
    if (out->prec != in->prec || out->nrhs != in->nrhs) fail(MSPCG_EINVAL, "m5inv: precision/nrhs mismatch");
    Op5Args a;
    std::memset(&a, 0, sizeof(a));
    a.nsites = h->Vh;
    a.Ls = h->par.Ls;
    a.nrhs = in->nrhs;
    a.nsite_wg = pick_nsite(in->nrhs, h->par.Ls);
    a.in = in->data;
    a.in_norm = in->norm;
    a.out = out->data;
    a.out_norm = out->norm;
    a.stride = h->Vh;
    a.inv = 1;
    a.dag = dagger ? 1 : 0;
    a.chain = h->m5inv.ptr(in->prec);
    HIPCHK(launch_op5(in->prec, a, S(stream)));
  });
}

mspcg_status mdagm(mspcg_handle *h, mspcg_field *out, const mspcg_field *in, void *stream) {
  return guarded([&] {
    if (!h) fail(MSPCG_EINVAL, "NULL handle");
    check_field(h, out, "out");
    check_field(h, in, "in");
    if (out->parity != 0 || in->parity != 0) fail(MSPCG_EINVAL, "mdagm acts on even fields");
    if (out->prec != in->prec || out->nrhs != in->nrhs) fail(MSPCG_EINVAL, "mdagm: precision/nrhs mismatch");
    if (out->data == in->data) fail(MSPCG_EINVAL, "mdagm: out must not alias in");
    const int prec = in->prec, nrhs = in->nrhs;
    h->tmp_o2.ensure(prec, nrhs, h->Vh, h->par.Ls);
    h->tmp_e2.ensure(prec, nrhs, h->Vh, h->par.Ls);
    apply_mdagm(h, prec, nrhs, vec_of(h, out), vec_of(h, in), h->tmp_o2.v, h->tmp_e2.v, nullptr, S(stream));
  });
}

mspcg_status mdagm_noalloc(mspcg_handle *h, mspcg_field *out, const mspcg_field *in, void *stream) {
  return guarded([&] {
    if (!h) fail(MSPCG_EINVAL, "NULL handle");
    check_field(h, out, "out");
    check_field(h, in, "in");
    if (out->parity != 0 || in->parity != 0) fail(MSPCG_EINVAL, "mdagm_noalloc acts on even fields");
    if (out->prec != in->prec || out->nrhs != in->nrhs) fail(MSPCG_EINVAL, "mdagm_noalloc: precision/nrhs mismatch");
    if (out->data == in->data) fail(MSPCG_EINVAL, "mdagm_noalloc: out must not alias in");
    const int prec = in->prec, nrhs = in->nrhs, Ls = h->par.Ls;
    if (!h->links_ok[prec])
      fail(MSPCG_EUNSUPPORTED, "mdagm_noalloc: links of this precision not prepared (call an operator in it first)");
    // two intermediate fields (odd, even), each with its norms, 256-byte aligned
    auto align = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t n5 = (size_t)nrhs * h->Vh * Ls;
    const size_t data_b = align(n5 * 24 * prec_bytes(prec));
    const size_t norm_b = prec_norm(prec) ? align(n5 * sizeof(float)) : 0;
    const size_t need = 2 * (data_b + norm_b);
    if (need > (size_t)MSPCG_NOALLOC_SCRATCH_BYTES)
      fail(MSPCG_EUNSUPPORTED, "mdagm_noalloc: the two intermediate fields need " + std::to_string(need) +
                                   " bytes, above MSPCG_NOALLOC_SCRATCH_BYTES = " +
                                   std::to_string((size_t)MSPCG_NOALLOC_SCRATCH_BYTES));
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev != h->device) fail(MSPCG_EINVAL, "mdagm_noalloc: the current device is not the handle's device");
    unsigned char *base = static_cast<unsigned char *>(h->scratch_dev);
    Vec to, te;
    to.prec = te.prec = prec;
    to.stride = te.stride = h->Vh;
    to.data = base;
    to.norm = norm_b ? reinterpret_cast<float *>(base + data_b) : nullptr;
    te.data = base + data_b + norm_b;
    te.norm = norm_b ? reinterpret_cast<float *>(base + 2 * data_b + norm_b) : nullptr;
    apply_mdagm(h, prec, nrhs, vec_of(h, out), vec_of(h, in), to, te, nullptr, S(stream), /*may_tune=*/false);
  });
}

mspcg_status local_block_cg(mspcg_handle *h, mspcg_field *z, const mspcg_field *r, const mspcg_precond *pc,
                            void *stream) {
  return guarded([&] {
    if (!h || !pc) fail(MSPCG_EINVAL, "NULL handle or preconditioner");
    check_field(h, z, "z");
    check_field(h, r, "r");
    if (z->prec != r->prec) fail(MSPCG_EINVAL, "local_block_cg: r and z differ in precision");
    if (z->prec != MSPCG_F64 && z->prec != MSPCG_F32) fail(MSPCG_EUNSUPPORTED, "local_block_cg takes F64 or F32 r and z");
    if (z->parity != 0 || r->parity != 0) fail(MSPCG_EINVAL, "local_block_cg works on even sites");
    if (z->nrhs != r->nrhs) fail(MSPCG_EINVAL, "nrhs mismatch");
    if (z->data == r->data) fail(MSPCG_EINVAL, "local_block_cg: z must not alias r");
    if (pc->n_inner < 0) fail(MSPCG_EINVAL, "n_inner < 0");
    if (pc->inner_prec < MSPCG_F64 || pc->inner_prec > MSPCG_BF16) fail(MSPCG_EINVAL, "bad inner precision");
    if (!(pc->inner_tol >= 0.0) || !std::isfinite(pc->inner_tol)) fail(MSPCG_EINVAL, "inner_tol < 0 or not finite");
    if (pc->n_sweeps < 0) fail(MSPCG_EINVAL, "n_sweeps < 0");
    hipStream_t st = S(stream);
    BlockGeom *bg = get_blocks(h, pc->nblk, pc->no_snake, st);
    const int nrhs = r->nrhs;
    const long long n = (long long)h->Vh * h->par.Ls * 24;
    ensure_block_vecs(h, bg, pc->inner_prec, nrhs);
    h->partial.ensure((size_t)std::max(kBlasGrid, bg->be_tot) * nrhs * sizeof(double));
    // F32 boundary fields: the preconditioner works on F64 copies
    Vec Zv = vec_of(h, z), Rv = vec_of(h, r);
    if (r->prec == MSPCG_F32) {
      h->lbc_r.ensure(MSPCG_F64, nrhs, h->Vh, h->par.Ls);
      h->lbc_z.ensure(MSPCG_F64, nrhs, h->Vh, h->par.Ls);
      HIPCHK(launch_convert(h->lbc_r.v, Rv, nrhs, (long long)h->Vh * h->par.Ls, h->par.Ls, st));
      Rv = h->lbc_r.v;
      Zv = h->lbc_z.v;
    }
    double *rr = bg->rrbuf.as<double>();
    HIPCHK(blas_dot_partial((const double *)Rv.data, (const double *)Rv.data, n, nrhs, h->partial.as<double>(), st));
    HIPCHK(blas_reduce(h->partial.as<double>(), kBlasGrid, nrhs, rr, st));
    run_block_cg(h, bg, pc->inner_prec, nrhs, pc->n_inner, pc->inner_tol, Zv, Rv, rr, nullptr, nullptr, st);
    if (pc->n_sweeps > 1) {
      h->scal.ensure((size_t)nrhs * 11 * sizeof(double) + 64);
      more_sweeps(h, nrhs, pc->n_sweeps, Zv, Rv, h->scal.as<double>(), h->partial.as<double>(), st,
                  [&](const Vec &z2, const Vec &t, double *rrt) {
                    run_block_cg(h, bg, pc->inner_prec, nrhs, pc->n_inner, pc->inner_tol, z2, t, rrt, nullptr,
                                 nullptr, st);
                  });
    }
    if (z->prec == MSPCG_F32)
      HIPCHK(launch_convert(vec_of(h, z), Zv, nrhs, (long long)h->Vh * h->par.Ls, h->par.Ls, st));
  });
}

mspcg_status cg_solve(mspcg_handle *h, mspcg_field *x, const mspcg_field *b, const mspcg_solver *s,
                      mspcg_stats *st) {
  return solve(h, x, b, s, nullptr, st);
}

mspcg_status mspcg_solve(mspcg_handle *h, mspcg_field *x, const mspcg_field *b, const mspcg_solver *s,
                         const mspcg_precond *pc, mspcg_stats *st) {
  if (!pc) {
    g_last_error = "NULL preconditioner";
    return MSPCG_EINVAL;
  }
  return solve(h, x, b, s, pc, st);
}

mspcg_status dwf_prepare_rhs(mspcg_handle *h, mspcg_field *b, const mspcg_field *phi_e, const mspcg_field *phi_o,
                             void *stream) {
  return guarded([&] {
    if (!h) fail(MSPCG_EINVAL, "NULL handle");
    check_field(h, b, "b");
    check_field(h, phi_e, "phi_e");
    check_field(h, phi_o, "phi_o");
    if (b->prec != MSPCG_F64 || phi_e->prec != MSPCG_F64 || phi_o->prec != MSPCG_F64)
      fail(MSPCG_EINVAL, "dwf_prepare_rhs takes F64 fields");
    if (b->parity != 0 || phi_e->parity != 0 || phi_o->parity != 1) fail(MSPCG_EINVAL, "parity mismatch");
    const int nrhs = b->nrhs;
    if (phi_e->nrhs != nrhs || phi_o->nrhs != nrhs) fail(MSPCG_EINVAL, "nrhs mismatch");
    hipStream_t st = S(stream);
    ensure_fp64_temps(h, nrhs);
    const long long n = (long long)h->Vh * h->par.Ls * 24;
    const Vec to = h->tmp_o.v, te = h->tmp_e.v;
    // t_o = M_5^{-1} phi_o
    Op5Args a;
    std::memset(&a, 0, sizeof(a));
    a.nsites = h->Vh;
    a.Ls = h->par.Ls;
    a.nrhs = nrhs;
    a.nsite_wg = pick_nsite(nrhs, h->par.Ls);
    a.in = phi_o->data;
    a.out = to.data;
    a.stride = h->Vh;
    a.inv = 1;
    a.chain = h->m5inv.ptr(MSPCG_F64);
    HIPCHK(launch_op5(MSPCG_F64, a, st));
    // te = M^4_eo t_o ; phihat = phi_e - te (into te)
    global_hop(h, MSPCG_F64, nrhs, 0, te, to, 0, 1, EPI_SCALE, -0.5, nullptr, nullptr, nullptr, nullptr, st);
    HIPCHK(blas_axpby((double *)te.data, 1.0, (const double *)phi_e->data, -1.0, (const double *)te.data, n, nrhs, st));
    // b = D_PC^+ phihat
    global_hop(h, MSPCG_F64, nrhs, 1, to, te, 1, 0, EPI_M5INV, -0.5, &h->x1, nullptr, nullptr, nullptr,
               st);
    global_hop(h, MSPCG_F64, nrhs, 0, vec_of(h, b), to, 1, 0, EPI_M5DAG_MPHIDAG, 0.5, nullptr, &te, nullptr, nullptr,
               st);
    HIPCHK(hipStreamSynchronize(st));
  });
}

mspcg_status dwf_reconstruct(mspcg_handle *h, mspcg_field *psi_o, const mspcg_field *psi_e, const mspcg_field *phi_o,
                             void *stream) {
  return guarded([&] {
    if (!h) fail(MSPCG_EINVAL, "NULL handle");
    check_field(h, psi_o, "psi_o");
    check_field(h, psi_e, "psi_e");
    check_field(h, phi_o, "phi_o");
    if (psi_o->prec != MSPCG_F64 || psi_e->prec != MSPCG_F64 || phi_o->prec != MSPCG_F64)
      fail(MSPCG_EINVAL, "dwf_reconstruct takes F64 fields");
    if (psi_o->parity != 1 || psi_e->parity != 0 || phi_o->parity != 1) fail(MSPCG_EINVAL, "parity mismatch");
    const int nrhs = psi_o->nrhs;
    if (psi_e->nrhs != nrhs || phi_o->nrhs != nrhs) fail(MSPCG_EINVAL, "nrhs mismatch");
    hipStream_t st = S(stream);
    ensure_fp64_temps(h, nrhs);
    const long long n = (long long)h->Vh * h->par.Ls * 24;
    const Vec to = h->tmp_o.v;
    // t = phi_o - M^4_oe psi_e ; psi_o = M_5^{-1} t
    global_hop(h, MSPCG_F64, nrhs, 1, to, vec_of(h, psi_e), 0, 1, EPI_SCALE, -0.5, nullptr, nullptr, nullptr, nullptr,
               st);
    HIPCHK(blas_axpby((double *)to.data, 1.0, (const double *)phi_o->data, -1.0, (const double *)to.data, n, nrhs, st));
    Op5Args a;
    std::memset(&a, 0, sizeof(a));
    a.nsites = h->Vh;
    a.Ls = h->par.Ls;
    a.nrhs = nrhs;
    a.nsite_wg = pick_nsite(nrhs, h->par.Ls);
    a.in = to.data;
    a.out = psi_o->data;
    a.stride = h->Vh;
    a.inv = 1;
    a.chain = h->m5inv.ptr(MSPCG_F64);
    HIPCHK(launch_op5(MSPCG_F64, a, st));
    HIPCHK(hipStreamSynchronize(st));
  });
}

mspcg_status mspcg_debug_site_maps(mspcg_handle *h, int parity, int32_t *lex_of_cb, int32_t *nbr) {
  return guarded([&] {
    if (!h || (parity & ~1)) fail(MSPCG_EINVAL, "bad handle or parity");
    if (lex_of_cb) std::memcpy(lex_of_cb, h->lex_of_cb[parity].data(), (size_t)h->Vh * sizeof(int32_t));
    if (nbr) std::memcpy(nbr, h->nbr_cb[parity].data(), (size_t)h->Vh * 8 * sizeof(int32_t));
  });
}

mspcg_status mspcg_debug_block_sites(mspcg_handle *h, const int nblk[4], int block, int32_t counts[3], int32_t *be_lex,
                                     int32_t *o1_lex, int32_t *e2_lex) {
  return guarded([&] {
    if (!h || !nblk || !counts) fail(MSPCG_EINVAL, "NULL argument");
    BlockGeom *bg = get_blocks(h, nblk, 0, h->stream);
    if (block < 0 || block >= bg->nb) fail(MSPCG_EINVAL, "block out of range");
    counts[0] = bg->be_n[block];
    counts[1] = bg->o1_n[block];
    counts[2] = bg->e2_n[block];
    if (be_lex) std::memcpy(be_lex, bg->be_lex.data() + bg->be_off[block], counts[0] * sizeof(int32_t));
    if (o1_lex) std::memcpy(o1_lex, bg->o1_lex.data() + bg->o1_off[block], counts[1] * sizeof(int32_t));
    if (e2_lex) std::memcpy(e2_lex, bg->e2_lex.data() + bg->e2_off[block], counts[2] * sizeof(int32_t));
  });
}

mspcg_status mspcg_block_apply(mspcg_handle *h, mspcg_field *out, const mspcg_field *in, const mspcg_precond *pc,
                               void *stream) {
  return guarded([&] {
    if (!h || !pc) fail(MSPCG_EINVAL, "NULL argument");
    check_field(h, out, "out");
    check_field(h, in, "in");
    if (out->prec != MSPCG_F64 || in->prec != MSPCG_F64) fail(MSPCG_EINVAL, "mspcg_block_apply takes F64 fields");
    if (out->parity != 0 || in->parity != 0) fail(MSPCG_EINVAL, "mspcg_block_apply works on even sites");
    if (out->nrhs != in->nrhs) fail(MSPCG_EINVAL, "nrhs mismatch");
    const int prec = pc->inner_prec;
    if (prec < MSPCG_F64 || prec > MSPCG_BF16) fail(MSPCG_EINVAL, "bad precision");
    if (out->data == in->data) fail(MSPCG_EINVAL, "out must not alias in");
    hipStream_t st = S(stream);
    BlockGeom *bg = get_blocks(h, pc->nblk, pc->no_snake, st);
    const int nrhs = in->nrhs;
    ensure_links(h, prec, st);
    ensure_block_vecs(h, bg, prec, nrhs);
    BlockArgs ba = block_args(h, bg, nrhs);
    const double n_total = (double)h->Vh * h->par.Ls * 24;
    double *part = bg->partial.as<double>();
    HIPCHK(block_gather(prec, ba, bg->x.v, bg->r.v, bg->p.v, bg->mp.v, vec_of(h, in), nullptr, n_total, part, st));
    (void)block_hops(h, bg, prec, nrhs, bg->p.v, bg->mp.v, bg->Ap.v, nullptr, st);
    HIPCHK(block_scatter(prec, ba, vec_of(h, out), bg->Ap.v, Vec(), nullptr, 0, Vec(), nullptr, n_total, part, st));
  });
}

mspcg_status mspcg_debug_block_hop(mspcg_handle *h, const mspcg_precond *pc, int nrhs, int hop, int reps,
                                   long long sites[2], void *stream) {
  return guarded([&] {
    if (!h || !pc) fail(MSPCG_EINVAL, "NULL argument");
    if (hop < 1 || hop > 4 || reps < 0) fail(MSPCG_EINVAL, "hop must be 1..4 and reps >= 0");
    if (nrhs < 1 || nrhs > MSPCG_MAX_NRHS) fail(MSPCG_EINVAL, "bad nrhs");
    const int prec = pc->inner_prec;
    if (prec < MSPCG_F64 || prec > MSPCG_BF16) fail(MSPCG_EINVAL, "bad precision");
    if (hop_threads(h->par.Ls, nrhs, 1) > 256) fail(MSPCG_EUNSUPPORTED, "nrhs x Ls above one workgroup");
    hipStream_t st = S(stream);
    BlockGeom *bg = get_blocks(h, pc->nblk, pc->no_snake, st);
    ensure_links(h, prec, st);
    ensure_block_vecs(h, bg, prec, nrhs);
    double *part = bg->partial.as<double>();
    // (as the fixed-k solve launches them: with the snake terms the second hop
    // forms the <p, A_s p> partials and the last updates r in place with the
    // |r|^2 partials; without them the last forms the <p, A_s p> partials)
    const bool upd = hop == 4 && !bg->no_snake;
    const int dot_hop = bg->no_snake ? 4 : 2;
    for (int i = 0; i < reps; ++i)
      block_hop(h, bg, prec, nrhs, hop, bg->p.v, bg->mp.v, bg->Ap.v, (hop == dot_hop || upd) ? part : nullptr, st,
                upd ? bg->scal.as<double>() : nullptr);
    if (sites) {
      // input and output domains: 1: B_e -> O1, 2: O1 -> E2, 3: E2 -> O1, 4: O1 -> B_e
      long long nbe = 0, no1 = 0, ne2 = 0;
      for (int b = 0; b < bg->nb; ++b) nbe += bg->be_n[b], no1 += bg->o1_n[b], ne2 += bg->e2_n[b];
      sites[0] = hop == 1 ? nbe : hop == 3 ? ne2 : no1;
      sites[1] = hop == 2 ? ne2 : hop == 4 ? nbe : no1;
    }
  });
}

mspcg_status mspcg_convert(mspcg_handle *h, mspcg_field *out, const mspcg_field *in, void *stream) {
  return guarded([&] {
    if (!h) fail(MSPCG_EINVAL, "NULL handle");
    check_field(h, out, "out");
    check_field(h, in, "in");
    if (out->nrhs != in->nrhs || out->parity != in->parity) fail(MSPCG_EINVAL, "convert: nrhs/parity mismatch");
    HIPCHK(launch_convert(vec_of(h, out), vec_of(h, in), in->nrhs, (long long)h->Vh * h->par.Ls, h->par.Ls, S(stream)));
  });
}

}  // extern "C"
