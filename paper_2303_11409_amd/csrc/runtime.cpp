// Host runtime of the U(1)-symmetric MPS engine: the C ABI of u1mps.h.
//
// Per batch of gates (one brickwork layer, or a single gate) the runtime
//   1. enumerates the charge sectors on the host (integer bookkeeping:
//      middle charges m, Theta(m) shapes, (cL, cR) tiles with their cM
//      windows -- the "loop over allowed charge values" of Sec. II),
//   2. builds the gate blocks G^(n) from the 2x2 mode unitary,
//   3. uploads one packed work list and launches theta, Jacobi and select
//      kernels for all gates together,
//   4. reads back the kept count of every sector (the only host sync of the
//      batch), rebuilds the middle bonds' charge tables and launches the
//      update kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/u1mps.h"
#include "internal.h"
#include "kernels.h"

using namespace u1mps;

namespace {

thread_local std::string g_err = "no error";

mps_status fail(mps_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIPCHK(expr)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) return fail(MPS_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define STCHK(expr)                  \
  do {                               \
    mps_status s_ = (expr);          \
    if (s_ != MPS_OK) return s_;     \
  } while (0)

struct Bond {
  std::vector<int> charge;   // ascending
  std::vector<int> count;
  std::vector<int> off;      // prefix sums, size charge.size() + 1
  int dim() const { return off.empty() ? 0 : off.back(); }
  int find(int c) const {
    auto it = std::lower_bound(charge.begin(), charge.end(), c);
    return (it != charge.end() && *it == c) ? int(it - charge.begin()) : -1;
  }
  int lower(int c) const { return int(std::lower_bound(charge.begin(), charge.end(), c) - charge.begin()); }
  void finish() {
    off.assign(charge.size() + 1, 0);
    for (size_t i = 0; i < charge.size(); ++i) off[i + 1] = off[i] + count[i];
  }
};

// Charge arithmetic: U(1) (mod 0) or Z_n (mod n, charges in 0..n-1).
inline int cwrap(int mod, int c) { return mod ? ((c % mod) + mod) % mod : c; }

// The charge rule of a state.  Local state p carries the charge step[p]; an
// entry of a site tensor between left charge cL and right charge cR is allowed
// when cL - cR is some step[p] (mod n for Z_n), and then p is its local state:
// Eq. (E2), with the occupation in the Kronecker delta replaced by the local
// state's charge.  U(1) photon number: step[p] = p.  Z_n (d <= n): the same
// steps, charges mod n.  Two U(1) charges (the general Abelian case): a charge
// (c1, c2) is the integer key c1 * radix + c2 with radix above twice every
// second component, so keys add like the pairs, a difference of keys fixes
// the difference of pairs, and ascending keys are the pairs in lexicographic
// order; step[p] is the key of local state p's pair.
struct ChargeRule {
  int mod = 0;
  std::vector<int> step;      // d entries, distinct, >= 0
  std::vector<int> sums;      // distinct two-site totals step[p] + step[q] (mod n), ascending
  int minstep = 0, maxstep = 0;
  bool photon = true;         // U(1) with step[p] = p (beam splitters apply)
  void init(int m, const std::vector<int>& st) {
    mod = m;
    step = st;
    const int d = (int)st.size();
    photon = !m;
    for (int p = 0; p < d; ++p) photon = photon && st[p] == p;
    minstep = *std::min_element(st.begin(), st.end());
    maxstep = *std::max_element(st.begin(), st.end());
    sums.clear();
    for (int p = 0; p < d; ++p)
      for (int q = 0; q < d; ++q) sums.push_back(cwrap(m, st[p] + st[q]));
    std::sort(sums.begin(), sums.end());
    sums.erase(std::unique(sums.begin(), sums.end()), sums.end());
  }
  // the local state p with step[p] == diff (mod n), or -1
  int local(int diff) const {
    if (mod) diff = cwrap(mod, diff);
    for (size_t p = 0; p < step.size(); ++p)
      if (step[p] == diff) return (int)p;
    return -1;
  }
  bool ok(int ci, int cj) const { return local(ci - cj) >= 0; }
  int sum_index(int total) const {
    if (mod) total = cwrap(mod, total);
    auto it = std::lower_bound(sums.begin(), sums.end(), total);
    return (it != sums.end() && *it == total) ? int(it - sums.begin()) : -1;
  }
  // does a two-site element (p, q) <- (a, b) keep the charge?
  bool conserves(int p, int q, int a, int b) const {
    return cwrap(mod, step[p] + step[q] - step[a] - step[b]) == 0;
  }
};

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
};

struct PinBuf {
  void* p = nullptr;
  size_t cap = 0;
};

enum Kind { K_THETA = 0, K_SELECT, K_UPDATE, K_JACOBI, K_JACOBI8, K_JACOBI_AUX, K_GEMM, K_SPLIT };

struct Pending {
  int kind;
  hipEvent_t a, b;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Rotation sweeps over a block pair's Gram matrix before the block is rotated
// (per pass).  The outer sweeps carry convergence: the Gram of a block pair
// need not be diagonalised before its vectors are rotated, and one inner sweep
// per visit costs ~19 % more outer sweeps but far less eig time per launch
// (the eig's sequential rotation steps bound the launch).
constexpr int kMaxInnerSweeps = 1;
// Blocked sweeps before an unconverged sector is finished by scalar sweeps.
constexpr int kBlockedSweeps = 32;
// Desynchronised sweeps: launches between reads of the count of sectors
// still sweeping.
constexpr int kDesyncCheck = 16;

}  // namespace

struct mps_state {
  int L = 0, d = 0, N = 0;
  int mod = 0;                   // 0: U(1) particle number; n: particle number mod n (d <= n)
  int device = 0;                // the GPU current when the handle was created
  int cus = 256;                 // compute units of that GPU
  ChargeRule rule;               // charges of the local states (U(1), Z_n, or two U(1) components)
  int ncomp = 1;                 // charge components packed into one key (1 or 2)
  int radix = 0;                 // ncomp == 2: key = c1 * radix + c2
  mps_opts opts{};
  mps_device dev{};
  hipStream_t st = nullptr;
  hipStream_t cap_st = nullptr;  // private stream for graph capture (the handle's may be the null stream)
  std::vector<Bond> bonds;       // L + 1
  std::vector<int> cap;          // per bond: largest admissible dimension
  std::vector<double*> lam;      // per bond, cap[b] doubles
  std::vector<double2*> site;    // per site, cap[s] * cap[s+1] complex
  // workspaces (grow-only)
  DevBuf th_raw, th_scaled, acc, sigma, order, jperm, jnorm, plan, upd, norm_e0, norm_e1, norm_t, sel_v, sel_k, misc,
      pbuf, planes, envs, samp, tbefore;
  std::vector<double> last_leak;   // per gate of the last apply call touching this state
  PinBuf stage_plan, stage_upd, stage_res, stage_misc, stage_flag, stage_samp;
  mps_stats stats{};
  bool timing = false;
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
};

namespace {

void* dalloc(mps_state* h, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (h->dev.alloc) return h->dev.alloc(bytes, h->dev.ctx);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  return p;
}

void dfree(mps_state* h, void* p) {
  if (!p) return;
  if (h->dev.release) h->dev.release(p, h->dev.ctx);
  else (void)hipFree(p);
}

mps_status ensure(mps_state* h, DevBuf& b, size_t bytes) {
  if (b.cap >= bytes) return MPS_OK;
  size_t nb = std::max(bytes, b.cap + b.cap / 2);
  nb = align256(nb);
  if (b.p) {
    HIPCHK(hipStreamSynchronize(h->st));
    dfree(h, b.p);
    b.p = nullptr;
    b.cap = 0;
  }
  void* p = dalloc(h, nb);
  if (!p) return fail(MPS_E_NOMEM, "device allocation of %zu bytes failed", nb);
  b.p = p;
  b.cap = nb;
  return MPS_OK;
}

mps_status ensure_pin(PinBuf& b, size_t bytes) {
  if (b.cap >= bytes) return MPS_OK;
  size_t nb = align256(std::max(bytes, b.cap + b.cap / 2));
  if (b.p) {
    (void)hipHostFree(b.p);
    b.p = nullptr;
    b.cap = 0;
  }
  void* p = nullptr;
  if (hipHostMalloc(&p, nb, hipHostMallocDefault) != hipSuccess || !p)
    return fail(MPS_E_NOMEM, "pinned host allocation of %zu bytes failed", nb);
  b.p = p;
  b.cap = nb;
  return MPS_OK;
}

// Packs several host arrays into one pinned block; offsets are 256-aligned.
struct Packer {
  struct Item {
    const void* src;
    size_t bytes;
    size_t off;
  };
  std::vector<Item> items;
  size_t total = 0;
  size_t add(const void* src, size_t bytes) {
    const size_t off = total;
    items.push_back({src, bytes, off});
    total = align256(total + std::max<size_t>(bytes, 1));
    return off;
  }
  // Copies the items that have a source; items added with src == nullptr are
  // device-side outputs and only reserve space.
  void write(void* dst) const {
    for (const Item& it : items)
      if (it.src && it.bytes) std::memcpy(static_cast<char*>(dst) + it.off, it.src, it.bytes);
  }
};

template <class T>
T* at(const DevBuf& b, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(b.p) + off);
}

// ---- timing ----------------------------------------------------------------
mps_status ev_get(mps_state* h, hipEvent_t* e) {
  if (!h->pool.empty()) {
    *e = h->pool.back();
    h->pool.pop_back();
    return MPS_OK;
  }
  HIPCHK(hipEventCreate(e));
  return MPS_OK;
}

struct Timer {
  mps_state* h;
  int kind;
  hipEvent_t a = nullptr, b = nullptr;
  bool on = false;
  Timer(mps_state* hh, int k) : h(hh), kind(k) {}
  mps_status start() {
    if (!h->timing) return MPS_OK;
    STCHK(ev_get(h, &a));
    STCHK(ev_get(h, &b));
    HIPCHK(hipEventRecord(a, h->st));
    on = true;
    return MPS_OK;
  }
  mps_status stop() {
    if (!on) return MPS_OK;
    HIPCHK(hipEventRecord(b, h->st));
    h->pending.push_back({kind, a, b});
    on = false;
    return MPS_OK;
  }
};

// Called after a stream synchronisation: fold finished event pairs into stats.
mps_status drain_events(mps_state* h) {
  for (const Pending& p : h->pending) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, p.a, p.b));
    switch (p.kind) {
      case K_THETA: h->stats.theta_ms += ms; break;
      case K_SELECT: h->stats.select_ms += ms; break;
      case K_JACOBI: h->stats.jacobi_ms += ms; break;
      case K_JACOBI8:
        h->stats.jacobi_ms += ms;
        h->stats.jacobi8_ms += ms;
        break;
      case K_JACOBI_AUX: h->stats.jacobi_aux_ms += ms; break;
      case K_GEMM: h->stats.gemm_ms += ms; break;
      case K_SPLIT: h->stats.split_ms += ms; break;
      default: h->stats.update_ms += ms; break;
    }
    h->pool.push_back(p.a);
    h->pool.push_back(p.b);
  }
  h->pending.clear();
  return MPS_OK;
}

// ---- gate blocks -----------------------------------------------------------
// G^(n)[p][a] = <p, n-p| G |a, n-a>.  The input state |a, b> is
// (a0^+)^a (a1^+)^b / sqrt(a! b!) |0>; substituting a0^+ -> u00 X + u10 Y and
// a1^+ -> u01 X + u11 Y and expanding the product as a polynomial in X (the
// power of Y is fixed by the degree), the coefficient of X^p Y^(n-p) times
// sqrt(p! (n-p)!) is the element.  Occupations >= d are dropped (cutoff).
void gate_blocks(const mps_z u[4], int d, double2* out) {
  using C = std::complex<double>;
  const C u00(u[0].re, u[0].im), u01(u[1].re, u[1].im), u10(u[2].re, u[2].im), u11(u[3].re, u[3].im);
  double fact[2 * kMaxD + 2];
  fact[0] = 1.0;
  for (int i = 1; i < 2 * kMaxD + 2; ++i) fact[i] = fact[i - 1] * i;
  const int nb = 2 * d - 1;
  for (int i = 0; i < nb * d * d; ++i) out[i] = make_double2(0.0, 0.0);
  for (int n = 0; n < nb; ++n) {
    for (int a = std::max(0, n - d + 1); a <= std::min(d - 1, n); ++a) {
      const int b = n - a;
      std::vector<C> poly(1, C(1.0, 0.0));
      auto mulf = [&](C cx, C cy) {       // poly *= (cx X + cy Y)
        std::vector<C> nx(poly.size() + 1, C(0.0, 0.0));
        for (size_t k = 0; k < poly.size(); ++k) {
          nx[k] += cy * poly[k];
          nx[k + 1] += cx * poly[k];
        }
        poly.swap(nx);
      };
      for (int i = 0; i < a; ++i) mulf(u00, u10);
      for (int i = 0; i < b; ++i) mulf(u01, u11);
      for (int p = std::max(0, n - d + 1); p <= std::min(d - 1, n); ++p) {
        const C v = poly[p] * std::sqrt(fact[p] * fact[n - p] / (fact[a] * fact[b]));
        out[(n * d + p) * d + a] = make_double2(v.real(), v.imag());
      }
    }
  }
}

// G^(n)[p][a] of a gate given as a dense d^2 x d^2 matrix (row p*d+q, column
// a*d+b): for the n-th two-site total S of the rule, the element of row
// p*d+q and column a*d+b with step[p] + step[q] = step[a] + step[b] = S (mod n
// for Z_n).  Elements that change the charge were checked to be negligible
// and are not read.
void dense_blocks(const mps_z* g4, int d, const ChargeRule& R, double2* out) {
  const int nb = (int)R.sums.size(), dd = d * d;
  for (int i = 0; i < nb * d * d; ++i) out[i] = make_double2(0.0, 0.0);
  for (int n = 0; n < nb; ++n) {
    const int S = R.sums[n];
    for (int p = 0; p < d; ++p) {
      const int q = R.local(S - R.step[p]);
      if (q < 0) continue;
      for (int a = 0; a < d; ++a) {
        const int b = R.local(S - R.step[a]);
        if (b < 0) continue;
        const mps_z v = g4[(size_t)(p * d + q) * dd + a * d + b];
        out[(n * d + p) * d + a] = make_double2(v.re, v.im);
      }
    }
  }
}

// ---- capacities ------------------------------------------------------------
// Largest Schmidt rank a bond can reach: sum over charges c of
// min(#left strings of total charge N - c, #right strings of total charge c),
// strings over the sites of each side with local states 0..d-1 (charges as
// keys 0..N, or mod n).
std::vector<double> strings_by_charge(int sites, const ChargeRule& R, int N) {
  const int n = R.mod ? R.mod : N + 1;
  std::vector<double> cnt(n, 0.0), nx(n);
  cnt[0] = 1.0;
  for (int s = 0; s < sites; ++s) {
    std::fill(nx.begin(), nx.end(), 0.0);
    for (int c = 0; c < n; ++c) {
      if (cnt[c] == 0.0) continue;
      for (int st : R.step) {
        const int c2 = R.mod ? (c + st) % R.mod : c + st;
        if (c2 < n) nx[c2] += cnt[c];
      }
    }
    cnt.swap(nx);
  }
  return cnt;
}

mps_status compute_caps(mps_state* h) {
  h->cap.assign(h->L + 1, 1);
  const int n = h->mod ? h->mod : h->N + 1;
  for (int b = 0; b <= h->L; ++b) {
    double tot = 0.0;
    const std::vector<double> left = strings_by_charge(b, h->rule, h->N);
    const std::vector<double> right = strings_by_charge(h->L - b, h->rule, h->N);
    for (int c = 0; c < n; ++c) {
      const int lc = h->mod ? cwrap(h->mod, h->N - c) : h->N - c;
      tot += std::min(left[lc], right[c]);
    }
    if (h->opts.chi_max > 0) tot = std::min(tot, double(h->opts.chi_max));
    tot = std::max(tot, double(h->bonds[b].dim()));
    if (tot > 65536.0)
      return fail(MPS_E_ARG, "bond %d could reach dimension %.3g; set chi_max", b, tot);
    h->cap[b] = std::max(1, int(tot));
  }
  return MPS_OK;
}

// ---- batch plan ------------------------------------------------------------
struct GatePlan {
  int site;
  int sec_begin, sec_end;
};

struct BatchPlan {
  std::vector<GateWork> gates;
  std::vector<SectorWork> secs;
  std::vector<ThetaTile> tiles;
  std::vector<double2> coef;
  std::vector<GatePlan> gp;
  std::vector<int> jlist;                 // every sector id
  std::vector<JacobiPairWork> jpairlist;  // every block pair of a step, heaviest sector first
  std::vector<int> jnb;                   // block count per jlist entry
  int jpairs = 0, jmaxnb = 2, jmaxrows = 1;
  int jblock = kJB8;                      // vectors per Jacobi block (8 or 16)
  std::vector<long long> sel_off;         // global sort scratch offsets
  long long sel_scratch = 0;
  int maxP = 1;
  long long th_elems = 0;
  long long acc_elems = 0;
  int sig_elems = 0;
  int maxw = 1;
  double theta_flops = 0.0;
  // split-BF16 form: the BF16 planes of every gate's two site tensors, then
  // one product per charge triple into the complex128 scratch
  bool split = false;
  std::vector<SplitPlanes> spl;
  std::vector<int> ktab;                  // padded k -> source k (-1 = pad), all gates
  int spl_tiles = 0;
  long long plane_elems = 0;
  std::vector<SplitGemm> sg;              // a, b, c hold buffer offsets until upload
  int sg_tiles[kSgVariants] = {0, 0, 0, 0};
  long long p_elems = 0;
  double sg_mfma_flops[kSgVariants] = {0.0, 0.0, 0.0, 0.0};
};

// One two-site update of a batch: the state it acts on, its left site and
// either its 2x2 mode unitary (u) or its dense d^2 x d^2 gate (g4, when u is
// NULL).  A batch may mix states (of one local dimension d).
struct GateRef {
  mps_state* h;
  int site;
  const mps_z* u;
  const mps_z* g4;
};

// Vectors per Jacobi block when the options leave it open.  A round-robin
// step lasts as long as its slowest block-pair visit, and a visit of 16
// vectors has about a quarter of the Gram and rotation work of a visit of 32
// and an eig of 15 steps instead of 31; but blocks of 8 double the steps of a
// sweep and the passes over the vectors.  Measured: blocks of 8 pay when the
// longest vectors are long (the 32-mode chi = 512 circuit, up to ~430
// elements: 0.755 s against 0.792 s) and the batch leaves room on the chip
// (fewer 32-vector block pairs than two per compute unit); with vectors of
// 256 (the Z_2 quench at chi = 256) or a full chip (batches of circuits, the
// chi = 2048 layer) blocks of 16 are faster.
int auto_jacobi_block(const std::vector<SectorWork>& secs, int cus) {
  long long pairs = 0;
  int maxlen = 0;
  for (const SectorWork& sw : secs) {
    int nb = (std::min(sw.r, sw.c) + kJB - 1) / kJB;
    nb += nb & 1;
    pairs += std::max(nb, 2) / 2;
    maxlen = std::max(maxlen, std::max(sw.r, sw.c));
  }
  return (maxlen >= 320 && pairs < 2LL * cus) ? kJB8 : kJB;
}

mps_status plan_batch(const std::vector<GateRef>& refs, BatchPlan& P) {
  const int ng = (int)refs.size();
  const int d = refs[0].h->d;
  P.split = refs[0].h->opts.form == MPS_FORM_SPLIT_BF16X3;
  P.jblock = refs[0].h->opts.jacobi_block;
  P.gates.resize(ng);
  P.gp.resize(ng);
  P.coef.clear();
  for (int g = 0; g < ng; ++g) {
    mps_state* h = refs[g].h;
    const ChargeRule& R = h->rule;
    const int s = refs[g].site;
    const Bond& BL = h->bonds[s];
    const Bond& BM = h->bonds[s + 1];
    const Bond& BR = h->bonds[s + 2];
    // gate blocks G^(n) for the rule's two-site totals (U(1): n = 0..2d-2)
    const size_t coef0 = P.coef.size();
    P.coef.resize(coef0 + R.sums.size() * d * d, make_double2(0.0, 0.0));
    double2* cg = P.coef.data() + coef0;
    if (refs[g].u)
      gate_blocks(refs[g].u, d, cg);
    else
      dense_blocks(refs[g].g4, d, R, cg);
    GateWork gw{};
    gw.bl = h->site[s];
    gw.br = h->site[s + 1];
    gw.lam_l = h->lam[s];
    gw.ldl = BM.dim();
    gw.ldr = BR.dim();
    gw.coef = (int)coef0;
    gw.d = d;
    gw.sec_begin = (int)P.secs.size();
    gw.keep_cap = h->cap[s + 1];
    gw.chi_max = h->opts.chi_max;
    gw.cutoff = h->opts.cutoff;
    gw.zero_tol = h->opts.zero_tol;
    // sectors: every middle charge m with rows (charges cL of bond s with
    // cL - m a local charge) and columns (charges cR of bond s+2 with m - cR a
    // local charge).  U(1): cL in [m, m+d-1], cR in [m-d+1, m]; Z_n: the same
    // mod n (with d = n every row and every column belongs to every m; with
    // d < n a range that wraps past n-1 is two blocks of the frame).  The rows of Theta(m)
    // are its row blocks in ascending charge order, packed; blocks adjacent
    // in the frame are merged (so a U(1) or Z_n sector is one row block and
    // one column block).
    const int zn = h->mod;
    std::vector<int> cand;
    if (zn) {
      for (int m = 0; m < zn; ++m) cand.push_back(m);
    } else {
      for (int cL : BL.charge)
        for (int st : R.step) cand.push_back(cL - st);
      std::sort(cand.begin(), cand.end());
      cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
    }
    std::vector<int> secm;          // middle charge of every sector of this gate, ascending
    int T = 0;
    auto add_block = [](int& nb, int* off, int* n, int* pos, int fo, int fn, int total) {
      if (nb > 0 && off[nb - 1] + n[nb - 1] == fo) {
        n[nb - 1] += fn;
      } else {
        off[nb] = fo;
        n[nb] = fn;
        pos[nb] = total;
        ++nb;
      }
    };
    for (int m : cand) {
      SectorWork sw{};
      int r = 0, c = 0;
      for (size_t i = 0; i < BL.charge.size(); ++i)
        if (R.ok(BL.charge[i], m)) {
          add_block(sw.nrb, sw.rb_off, sw.rb_n, sw.rb_pos, BL.off[i], BL.count[i], r);
          r += BL.count[i];
        }
      for (size_t j = 0; j < BR.charge.size(); ++j)
        if (R.ok(m, BR.charge[j])) {
          add_block(sw.ncb, sw.cb_off, sw.cb_n, sw.cb_pos, BR.off[j], BR.count[j], c);
          c += BR.count[j];
        }
      if (r <= 0 || c <= 0) continue;
      sw.gate = g;
      sw.m = m;
      sw.r = r;
      sw.c = c;
      sw.rlo = sw.rb_off[0];
      sw.clo = sw.cb_off[0];
      sw.off = P.th_elems;
      sw.sig = P.sig_elems;
      sw.kmax = std::min(r, c);
      sw.tall = r > c ? 1 : 0;
      sw.acc = P.acc_elems;
      if (sw.tall) P.acc_elems += (long long)c * c;
      secm.push_back(m);
      P.secs.push_back(sw);
      P.th_elems += (long long)r * c;
      P.sig_elems += r;
      T += sw.kmax;
    }
    auto sector_of = [&](int m) {
      auto it = std::lower_bound(secm.begin(), secm.end(), m);
      return (it != secm.end() && *it == m) ? gw.sec_begin + int(it - secm.begin()) : -1;
    };
    // position inside Theta(m) of frame row fr (resp. column fc)
    auto row_pos = [](const SectorWork& w, int fr) {
      for (int k = 0; k < w.nrb; ++k)
        if (fr >= w.rb_off[k] && fr < w.rb_off[k] + w.rb_n[k]) return w.rb_pos[k] + fr - w.rb_off[k];
      return -1;
    };
    auto col_pos = [](const SectorWork& w, int fc) {
      for (int k = 0; k < w.ncb; ++k)
        if (fc >= w.cb_off[k] && fc < w.cb_off[k] + w.cb_n[k]) return w.cb_pos[k] + fc - w.cb_off[k];
      return -1;
    };
    gw.sec_end = (int)P.secs.size();
    if (gw.sec_end == gw.sec_begin) return fail(MPS_E_CHARGE, "gate at site %d has no charge sector", s);
    if (gw.sec_end - gw.sec_begin > 1024) return fail(MPS_E_ARG, "more than 1024 sectors in one update");
    int Pp = 1;
    while (Pp < T) Pp <<= 1;
    P.maxP = std::max(P.maxP, Pp);
    P.sel_off.push_back(P.sel_scratch);
    P.sel_scratch += Pp;
    // split-BF16 form: planes of B[s] and of B[s+1] transposed over the middle
    // bond with every charge block padded to a multiple of 8
    std::vector<int> pm(BM.charge.size() + 1, 0);
    long long planeA = 0, planeB = 0;
    int ldk = 0;
    if (P.split) {
      for (size_t i = 0; i < BM.charge.size(); ++i) pm[i + 1] = pm[i] + ((BM.count[i] + 7) & ~7);
      ldk = pm.back();
      const long long k0 = (long long)P.ktab.size();
      for (size_t i = 0; i < BM.charge.size(); ++i)
        for (int t = 0; t < pm[i + 1] - pm[i]; ++t) P.ktab.push_back(t < BM.count[i] ? BM.off[i] + t : -1);
      const int tk = (ldk + kSpTile - 1) / kSpTile;
      SplitPlanes pa{gw.bl, gw.ldl, BL.dim(), 0, ldk, k0, P.plane_elems, tk, P.spl_tiles};
      planeA = P.plane_elems;
      P.plane_elems += (long long)kSgPlanes * BL.dim() * ldk;
      P.spl_tiles += ((BL.dim() + kSpTile - 1) / kSpTile) * tk;
      SplitPlanes pb{gw.br, gw.ldr, BR.dim(), 1, ldk, k0, P.plane_elems, tk, P.spl_tiles};
      planeB = P.plane_elems;
      P.plane_elems += (long long)kSgPlanes * BR.dim() * ldk;
      P.spl_tiles += ((BR.dim() + kSpTile - 1) / kSpTile) * tk;
      P.spl.push_back(pa);
      P.spl.push_back(pb);
    }
    // tiles
    gw.tile_begin = (int)P.tiles.size();
    for (size_t a = 0; a < BL.charge.size(); ++a) {
      const int cL = BL.charge[a];
      for (size_t b = 0; b < BR.charge.size(); ++b) {
        const int cR = BR.charge[b];
        const int n = R.sum_index(cL - cR);
        if (n < 0) continue;
        // the new sectors m (cL - m and m - cR local charges) and the old
        // middle charges cM (likewise), each in ascending charge order
        std::vector<std::pair<int, int>> outs, ins;
        for (int p = 0; p < d; ++p) {
          const int m = cwrap(zn, cL - R.step[p]);
          if (R.ok(m, cR)) outs.push_back({m, p});
        }
        std::sort(outs.begin(), outs.end());
        for (const auto& mp : outs) ins.push_back(mp);
        ThetaTile base{};
        base.gate = g;
        base.n = n;
        for (const auto& mp : outs) {
          const int si = sector_of(mp.first);
          if (si < 0) return fail(MPS_E_CHARGE, "internal: sector %d missing at site %d", mp.first, s);
          const SectorWork& sw = P.secs[si];
          base.sec[base.nout] = si;
          base.p[base.nout] = mp.second;
          base.orow[base.nout] = row_pos(sw, BL.off[a]);
          base.ocol[base.nout] = col_pos(sw, BR.off[b]);
          if (base.orow[base.nout] < 0 || base.ocol[base.nout] < 0)
            return fail(MPS_E_CHARGE, "internal: block outside sector %d at site %d", mp.first, s);
          ++base.nout;
        }
        int ksum = 0;
        int mid[kMaxD];
        for (const auto& mp : ins) {
          const int mi = BM.find(mp.first);
          if (mi < 0) continue;
          mid[base.nin] = mi;
          base.k0[base.nin] = BM.off[mi];
          base.kn[base.nin] = BM.count[mi];
          base.a[base.nin] = mp.second;
          ksum += BM.count[mi];
          ++base.nin;
        }
        P.maxw = std::max(P.maxw, base.nout);
        const int nL = BL.count[a], nR = BR.count[b];
        P.theta_flops += 8.0 * nL * double(ksum) * nR;
        if (P.split) {
          base.ldp = nR;
          for (int j = 0; j < base.nin; ++j) {
            base.poff[j] = P.p_elems;
            SplitGemm sg{};
            // offsets (elements) into the plane buffer and the scratch until upload
            sg.a = reinterpret_cast<const unsigned short*>(
                (uintptr_t)(planeA + (long long)BL.off[a] * ldk + pm[mid[j]]));
            sg.pa = (long long)BL.dim() * ldk;
            sg.lda = ldk;
            sg.b = reinterpret_cast<const unsigned short*>(
                (uintptr_t)(planeB + (long long)BR.off[b] * ldk + pm[mid[j]]));
            sg.pb = (long long)BR.dim() * ldk;
            sg.ldb = ldk;
            sg.c = reinterpret_cast<double2*>((uintptr_t)P.p_elems);
            sg.ldc = nR;
            sg.m = nL;
            sg.n = nR;
            sg.k = base.kn[j];
            for (int v = 0; v < kSgVariants; ++v) {
              const int tr = kSgTileR[v], tc = kSgTileC[v];
              sg.tiles_n[v] = (nR + tc - 1) / tc;
              sg.tile_begin[v] = P.sg_tiles[v];
              P.sg_tiles[v] += ((nL + tr - 1) / tr) * sg.tiles_n[v];
              // executed: whole tiles, k in steps of 16 (one MFMA k step)
              P.sg_mfma_flops[v] += 64.0 * tr * tc * 16.0 * (((nL + tr - 1) / tr) * sg.tiles_n[v]) *
                                    ((sg.k + 15) / 16);
            }
            P.sg.push_back(sg);
            P.p_elems += (long long)nL * nR;
          }
        }
        for (int ti = 0; ti < nL; ti += kThetaTile) {
          for (int tj = 0; tj < nR; tj += kThetaTile) {
            ThetaTile t = base;
            t.pr0 = ti;
            t.pc0 = tj;
            t.row0 = BL.off[a] + ti;
            t.nrow = std::min(kThetaTile, nL - ti);
            t.col0 = BR.off[b] + tj;
            t.ncol = std::min(kThetaTile, nR - tj);
            for (int i = 0; i < t.nout; ++i) {
              t.orow[i] += ti;
              t.ocol[i] += tj;
            }
            P.tiles.push_back(t);
          }
        }
      }
    }
    gw.tile_end = (int)P.tiles.size();
    P.gates[g] = gw;
    P.gp[g] = {s, gw.sec_begin, gw.sec_end};
  }
  // blocked Jacobi schedule: min(r, c) vectors in blocks of P.jblock, block
  // count even.  Block pairs are numbered heaviest sector first (longest vectors):
  // the dispatcher places workgroups in index order across the CUs, so the
  // slow pairs get a CU of their own and the light ones share.
  if (P.jblock == 0) P.jblock = auto_jacobi_block(P.secs, refs[0].h->cus);
  std::vector<int> jorder(P.secs.size());
  for (size_t i = 0; i < jorder.size(); ++i) jorder[i] = (int)i;
  std::stable_sort(jorder.begin(), jorder.end(), [&](int x, int y) {
    return std::max(P.secs[x].r, P.secs[x].c) > std::max(P.secs[y].r, P.secs[y].c);
  });
  for (int i : jorder) {
    const SectorWork& sw = P.secs[i];
    const int nv = std::min(sw.r, sw.c);
    int nb = (nv + P.jblock - 1) / P.jblock;
    nb += nb & 1;
    nb = std::max(nb, 2);
    P.jlist.push_back((int)i);
    P.jnb.push_back(nb);
    for (int k = 0; k < nb / 2; ++k) P.jpairlist.push_back({(int)i, nb, k, 0});
    P.jpairs += nb / 2;
    P.jmaxnb = std::max(P.jmaxnb, nb);
    P.jmaxrows = std::max(P.jmaxrows, nv);
  }
  return MPS_OK;
}

bool valid_handle(mps_t h) { return h != nullptr && h->L > 0; }

Steps steps_of(const mps_state* h) {
  Steps st{};
  for (int p = 0; p < h->d; ++p) st.s[p] = h->rule.step[p];
  return st;
}

mps_status check_device_limits(mps_state* h, const BatchPlan& P) {
  if ((size_t)P.jmaxrows * sizeof(double) > 64 * 1024)
    return fail(MPS_E_ARG, "sector with %d vectors exceeds the Jacobi sort and finalize LDS budget", P.jmaxrows);
  (void)h;
  return MPS_OK;
}

// ---- tile-shape tuner of the split-BF16 products ----------------------------
// The best output tile of the products depends on the charge-block sizes: the
// key of a batch is its histogram of products by the class of their row and
// column counts (up to 32, up to 64, more), each class weighted by its
// algorithmic flops and quantised to eighths.  The first batch with a key runs
// every tile shape once and keeps the fastest for that key for the rest of the
// process (all shapes give bitwise the same products).
std::mutex g_tile_mu;
std::map<std::string, int> g_tile_best;

std::string tile_key(const BatchPlan& P) {
  double w[9] = {0.0}, tot = 0.0;
  auto cls = [](int x) { return x <= 32 ? 0 : (x <= 64 ? 1 : 2); };
  for (const SplitGemm& g : P.sg) {
    const double f = double(g.m) * g.n * g.k;
    w[3 * cls(g.m) + cls(g.n)] += f;
    tot += f;
  }
  std::string key(9, '0');
  for (int i = 0; i < 9; ++i) key[i] = char('0' + (tot > 0.0 ? int(std::lround(8.0 * w[i] / tot)) : 0));
  return key;
}

bool tuned_variant(const std::string& key, int* v) {
  std::lock_guard<std::mutex> lk(g_tile_mu);
  auto it = g_tile_best.find(key);
  if (it == g_tile_best.end()) return false;
  *v = it->second;
  return true;
}

void remember_variant(const std::string& key, int v) {
  std::lock_guard<std::mutex> lk(g_tile_mu);
  g_tile_best[key] = v;
}

// ---- the batched two-site update ------------------------------------------
// The update of every gate in refs, all in one set of launches on the stream of
// refs[0]'s state, whose workspaces, timing and Jacobi options (max_sweeps,
// jacobi_tol) serve the whole batch.  Per-gate and per-sector statistics go
// to the state each gate belongs to.  No state changes unless every gate of
// the batch succeeds.
mps_status apply_batch(const std::vector<GateRef>& refs, double* discarded) {
  mps_state* h = refs[0].h;
  const int ng = (int)refs.size();
  using clock = std::chrono::steady_clock;
  auto plan_t0 = clock::now();
  auto plan_add = [&]() {
    h->stats.host_plan_ms += std::chrono::duration<double, std::milli>(clock::now() - plan_t0).count();
  };
  BatchPlan P;
  STCHK(plan_batch(refs, P));
  STCHK(check_device_limits(h, P));
  for (const GateRef& r : refs) r.h->stats.jacobi_block = P.jblock;
  const int ns = (int)P.secs.size();

  // workspaces
  STCHK(ensure(h, h->th_raw, (size_t)P.th_elems * sizeof(double2)));
  STCHK(ensure(h, h->th_scaled, (size_t)P.th_elems * sizeof(double2)));
  STCHK(ensure(h, h->acc, (size_t)std::max<long long>(P.acc_elems, 1) * sizeof(double2)));
  STCHK(ensure(h, h->sigma, (size_t)P.sig_elems * sizeof(double)));
  STCHK(ensure(h, h->order, (size_t)P.sig_elems * sizeof(int)));
  STCHK(ensure(h, h->jperm, (size_t)P.sig_elems * sizeof(int)));
  // two buffers of vector norms (one per sweep parity in desynchronised sweeps)
  STCHK(ensure(h, h->jnorm, 2 * (size_t)std::max<long long>(P.sig_elems, 1) * sizeof(double)));
  STCHK(ensure(h, h->tbefore, std::max<size_t>(P.tiles.size(), 1) * sizeof(double)));
  double* d_tbefore = static_cast<double*>(h->tbefore.p);
  if (P.split) {
    STCHK(ensure(h, h->pbuf, (size_t)std::max<long long>(P.p_elems, 1) * sizeof(double2)));
    STCHK(ensure(h, h->planes, (size_t)std::max<long long>(P.plane_elems, 1) * sizeof(unsigned short)));
    double2* pb = static_cast<double2*>(h->pbuf.p);
    const unsigned short* pl = static_cast<const unsigned short*>(h->planes.p);
    for (SplitGemm& g : P.sg) {
      g.a = pl + reinterpret_cast<uintptr_t>(g.a);
      g.b = pl + reinterpret_cast<uintptr_t>(g.b);
      g.c = pb + reinterpret_cast<uintptr_t>(g.c);
    }
  }
  const bool sel_global = P.maxP > kSelectLds || h->opts.select_scratch;
  if (sel_global) {
    STCHK(ensure(h, h->sel_v, (size_t)P.sel_scratch * sizeof(double)));
    STCHK(ensure(h, h->sel_k, (size_t)P.sel_scratch * sizeof(int)));
  }
  // packed work list
  Packer pk;
  const size_t o_gates = pk.add(P.gates.data(), P.gates.size() * sizeof(GateWork));
  const size_t o_secs = pk.add(P.secs.data(), P.secs.size() * sizeof(SectorWork));
  const size_t o_tiles = pk.add(P.tiles.data(), P.tiles.size() * sizeof(ThetaTile));
  const size_t o_coef = pk.add(P.coef.data(), P.coef.size() * sizeof(double2));
  const size_t o_jlist = pk.add(P.jlist.data(), P.jlist.size() * sizeof(int));
  const size_t o_jblk = pk.add(P.jpairlist.data(), P.jpairlist.size() * sizeof(JacobiPairWork));
  const size_t o_jnb = pk.add(P.jnb.data(), P.jnb.size() * sizeof(int));
  // desynchronised sweeps: sectors still sweeping (every sector with two or
  // more vectors), sectors stopped unconverged
  int ctr0[2] = {0, 0};
  for (const SectorWork& sw : P.secs) ctr0[0] += std::min(sw.r, sw.c) >= 2 ? 1 : 0;
  const size_t o_ctr = pk.add(ctr0, sizeof ctr0);
  const size_t o_seloff = pk.add(P.sel_off.data(), P.sel_off.size() * sizeof(long long));
  const size_t o_sg = pk.add(P.sg.data(), P.sg.size() * sizeof(SplitGemm));
  const size_t o_spl = pk.add(P.spl.data(), P.spl.size() * sizeof(SplitPlanes));
  const size_t o_ktab = pk.add(P.ktab.data(), P.ktab.size() * sizeof(int));
  const size_t o_kept = pk.add(nullptr, (size_t)ns * sizeof(int));
  const size_t o_cut = pk.add(nullptr, (size_t)ng * sizeof(CutOut));
  const size_t o_jst = pk.add(nullptr, (size_t)ns * sizeof(JacobiOut));
  const size_t o_active = pk.add(nullptr, 2 * sizeof(int));
  const size_t upload = o_kept;  // everything before the outputs is uploaded
  STCHK(ensure(h, h->plan, pk.total));
  STCHK(ensure_pin(h->stage_plan, upload));
  pk.write(h->stage_plan.p);
  HIPCHK(hipMemcpyAsync(h->plan.p, h->stage_plan.p, upload, hipMemcpyHostToDevice, h->st));
  plan_add();

  const GateWork* d_gates = at<GateWork>(h->plan, o_gates);
  const SectorWork* d_secs = at<SectorWork>(h->plan, o_secs);
  double2* raw = static_cast<double2*>(h->th_raw.p);
  double2* scaled = static_cast<double2*>(h->th_scaled.p);
  double* sig = static_cast<double*>(h->sigma.p);
  int* ord = static_cast<int*>(h->order.p);

  if (P.split) {
    {
      Timer tp(h, K_SPLIT);
      STCHK(tp.start());
      HIPCHK(launch_split_planes(at<SplitPlanes>(h->plan, o_spl), (int)P.spl.size(), P.spl_tiles,
                                 at<int>(h->plan, o_ktab), static_cast<unsigned short*>(h->planes.p), h->st));
      STCHK(tp.stop());
    }
    {
      const SplitGemm* d_sg = at<SplitGemm>(h->plan, o_sg);
      int variant = h->opts.tile_tuning >= 2 ? h->opts.tile_tuning - 2 : 0;
      bool have = h->opts.tile_tuning != 1;
      std::string key;
      if (!have) {
        key = tile_key(P);
        have = tuned_variant(key, &variant);
      }
      if (!have) {
        // first batch with this histogram: every tile shape once, timed; the
        // products are bitwise the same, so the last run's are kept
        hipEvent_t e0, e1;
        STCHK(ev_get(h, &e0));
        STCHK(ev_get(h, &e1));
        float best = 0.f;
        for (int v = 0; v < kSgVariants; ++v) {
          HIPCHK(hipEventRecord(e0, h->st));
          HIPCHK(launch_split_gemm(d_sg, (int)P.sg.size(), P.sg_tiles[v], v, h->st));
          HIPCHK(hipEventRecord(e1, h->st));
          HIPCHK(hipEventSynchronize(e1));
          float ms = 0.f;
          HIPCHK(hipEventElapsedTime(&ms, e0, e1));
          if (v == 0 || ms < best) {
            best = ms;
            variant = v;
          }
        }
        h->pool.push_back(e0);
        h->pool.push_back(e1);
        remember_variant(key, variant);
        h->stats.tile_tunings += 1;
      }
      Timer tg(h, K_GEMM);
      STCHK(tg.start());
      HIPCHK(launch_split_gemm(d_sg, (int)P.sg.size(), P.sg_tiles[variant], variant, h->st));
      STCHK(tg.stop());
      h->stats.gemm_launches += 1;
      h->stats.gemm_mfma_flops += P.sg_mfma_flops[variant];
      h->stats.gemm_variant = variant;
    }
    Timer tm(h, K_THETA);
    STCHK(tm.start());
    HIPCHK(launch_theta_mix(d_gates, at<ThetaTile>(h->plan, o_tiles), (int)P.tiles.size(), d_secs,
                            at<double2>(h->plan, o_coef), static_cast<const double2*>(h->pbuf.p), raw, scaled,
                            d_tbefore, h->st));
    STCHK(tm.stop());
  } else {
    Timer tm(h, K_THETA);
    STCHK(tm.start());
    HIPCHK(launch_theta(d_gates, at<ThetaTile>(h->plan, o_tiles), (int)P.tiles.size(), d_secs,
                        at<double2>(h->plan, o_coef), raw, scaled, d_tbefore, P.maxw, h->st));
    STCHK(tm.stop());
  }
  {
    JacobiOut* d_jst = at<JacobiOut>(h->plan, o_jst);
    const int* d_jlist = at<int>(h->plan, o_jlist);
    double2* d_acc = static_cast<double2*>(h->acc.p);
    int* d_perm = static_cast<int*>(h->jperm.p);
    double* d_norm = static_cast<double*>(h->jnorm.p);
    int* d_active = at<int>(h->plan, o_active);
    // two pinned slots for the per-sweep "still rotating" flag and largest
    // block count of the rotating sectors (see below)
    STCHK(ensure_pin(h->stage_flag, 4 * sizeof(int)));
    volatile int* flag = static_cast<volatile int*>(h->stage_flag.p);
    {
      Timer tm(h, K_JACOBI_AUX);
      STCHK(tm.start());
      HIPCHK(launch_jacobi_init(d_secs, d_jlist, ns, scaled, d_acc, d_jst, d_perm, d_norm, h->st));
      STCHK(tm.stop());
      h->stats.jacobi_aux_launches += 1;
    }
    // blocked sweeps; a sector still rotating after kBlockedSweeps of them is
    // finished by scalar sweeps on its vectors
    const int blocked =
        std::min(h->opts.max_sweeps, h->opts.blocked_sweeps > 0 ? h->opts.blocked_sweeps : kBlockedSweeps);
    // Sectors sweep at their own pace (below) unless lockstep is asked for, the
    // sweeps are replayed from a graph, or a sector has more vectors than a
    // workgroup's staging tiles hold for its norm sort.
    const bool desync = h->opts.jacobi_lockstep == 0 && !h->opts.sweep_graph &&
                        P.jmaxrows <= jacobi_desync_rows(P.jblock);
    // The step launches of a sweep are the same every sweep: with sweep_graph
    // they are captured once per update into a HIP graph and replayed on the
    // handle's stream.  Capture runs on a private stream (the null stream
    // cannot be captured); capturing executes nothing.
    struct GraphExec {
      hipGraphExec_t g = nullptr;
      ~GraphExec() {
        if (g) (void)hipGraphExecDestroy(g);
      }
    } gholder;
    hipGraphExec_t& gexec = gholder.g;
    if (h->opts.sweep_graph && P.jmaxnb > 1) {
      hipGraph_t graph = nullptr;
      if (!h->cap_st) HIPCHK(hipStreamCreateWithFlags(&h->cap_st, hipStreamNonBlocking));
      HIPCHK(hipStreamBeginCapture(h->cap_st, hipStreamCaptureModeThreadLocal));
      hipError_t ce = hipSuccess;
      for (int step = 0; step < P.jmaxnb - 1 && ce == hipSuccess; ++step)
        ce = launch_jacobi_step(d_secs, at<JacobiPairWork>(h->plan, o_jblk), P.jpairs, step, 0, blocked, nullptr,
                                scaled, d_acc, d_jst, d_perm, d_norm, 0, h->opts.jacobi_tol, kMaxInnerSweeps,
                                P.jblock, h->cap_st);
      const hipError_t ee = hipStreamEndCapture(h->cap_st, &graph);
      if (ce == hipSuccess) ce = ee;
      if (ce == hipSuccess) ce = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
      if (graph) (void)hipGraphDestroy(graph);
      if (ce != hipSuccess) return fail(MPS_E_DEVICE, "capture of the sweep graph failed: %s", hipGetErrorString(ce));
    }
    // The host never idles the device between sweeps: sweep k's flag (and the
    // largest block count of the sectors still rotating) is copied into
    // pinned slot k % 2 behind it, and the host reads it only once sweep
    // k + 1 is enqueued.  A sweep enqueued after convergence finds every
    // sector converged and returns at once, so it changes nothing.  Sweep
    // k + 2 launches only the steps of the sectors rotating after sweep k
    // (sectors only ever drop out, so those include every sector still
    // rotating then); a captured graph keeps the full count.
    hipEvent_t fev[2] = {nullptr, nullptr};
    STCHK(ev_get(h, &fev[0]));
    STCHK(ev_get(h, &fev[1]));
    int still_active = 1;
    if (desync) {
      // Every sector sweeps at its own pace: launch t runs each sector's step
      // t mod (nb - 1) of its sweep t div (nb - 1), the sweep ends folded
      // into the sweeps' first steps (jac_setup), so the launches number the
      // steps of the slowest sector rather than the sweeps of the slowest
      // times the steps of the largest.  Every kDesyncCheck launches the
      // count of sectors still sweeping is copied into a pinned slot behind
      // them; the host reads the previous copy, so it stays a few launches
      // ahead of the device, and stops once that count reads zero (launches
      // after that find every sector finished and return at once).
      int* d_ctr = at<int>(h->plan, o_ctr);
      const int tmax = blocked * (P.jmaxnb - 1) + 1;
      Timer tm(h, P.jblock == kJB8 ? K_JACOBI8 : K_JACOBI);
      STCHK(tm.start());
      int t = 0, checks = 0;
      bool over = false;
      while (t < tmax && !over) {
        HIPCHK(launch_jacobi_step(d_secs, at<JacobiPairWork>(h->plan, o_jblk), P.jpairs, t, 1, blocked, d_ctr,
                                  scaled, d_acc, d_jst, d_perm, d_norm, P.sig_elems, h->opts.jacobi_tol,
                                  kMaxInnerSweeps, P.jblock, h->st));
        ++t;
        if (t % kDesyncCheck == 0) {
          HIPCHK(hipMemcpyAsync(const_cast<int*>(flag) + 2 * (checks & 1), d_ctr, 2 * sizeof(int),
                                hipMemcpyDeviceToHost, h->st));
          HIPCHK(hipEventRecord(fev[checks & 1], h->st));
          if (checks >= 1) {
            HIPCHK(hipEventSynchronize(fev[(checks - 1) & 1]));
            if (flag[2 * ((checks - 1) & 1)] == 0) over = true;
          }
          ++checks;
        }
      }
      STCHK(tm.stop());
      h->stats.jacobi_launches += t;
      if (P.jblock == kJB8) h->stats.jacobi8_launches += t;
      // the counters after the last launch: every sector has finished (at
      // the latest at its step 0 of sweep `blocked`); still_active when one
      // stopped unconverged
      HIPCHK(hipMemcpyAsync(const_cast<int*>(flag) + 2 * (checks & 1), d_ctr, 2 * sizeof(int),
                            hipMemcpyDeviceToHost, h->st));
      HIPCHK(hipEventRecord(fev[checks & 1], h->st));
      HIPCHK(hipEventSynchronize(fev[checks & 1]));
      const volatile int* fl = flag + 2 * (checks & 1);
      if (fl[0] != 0) return fail(MPS_E_DEVICE, "%d Jacobi sectors still sweeping after the last step", fl[0]);
      still_active = fl[1] > 0 ? 1 : 0;
    } else {
      int issued = 0;
      int steps = P.jmaxnb - 1;
      for (int sweep = 0; sweep < blocked; ++sweep) {
        Timer tm(h, P.jblock == kJB8 ? K_JACOBI8 : K_JACOBI);
        STCHK(tm.start());
        int launched = P.jmaxnb - 1;
        if (gexec) {
          HIPCHK(hipGraphLaunch(gexec, h->st));
          h->stats.graph_launches += 1;
        } else {
          launched = steps;
          for (int step = 0; step < steps; ++step)
            HIPCHK(launch_jacobi_step(d_secs, at<JacobiPairWork>(h->plan, o_jblk), P.jpairs, step, 0, blocked,
                                      nullptr, scaled, d_acc, d_jst, d_perm, d_norm, 0, h->opts.jacobi_tol,
                                      kMaxInnerSweeps, P.jblock, h->st));
        }
        STCHK(tm.stop());
        h->stats.jacobi_launches += launched;
        if (P.jblock == kJB8) h->stats.jacobi8_launches += launched;
        Timer ta(h, K_JACOBI_AUX);
        STCHK(ta.start());
        HIPCHK(launch_jacobi_sweep_end(d_jlist, at<int>(h->plan, o_jnb), ns, d_jst, d_active, h->st));
        HIPCHK(launch_jacobi_sort(d_secs, d_jlist, ns, P.jmaxrows, d_jst, d_perm, d_norm, h->st));
        STCHK(ta.stop());
        h->stats.jacobi_aux_launches += 2;
        HIPCHK(hipMemcpyAsync(const_cast<int*>(flag) + 2 * (sweep & 1), d_active, 2 * sizeof(int),
                              hipMemcpyDeviceToHost, h->st));
        HIPCHK(hipEventRecord(fev[sweep & 1], h->st));
        issued = sweep + 1;
        if (sweep >= 1) {
          HIPCHK(hipEventSynchronize(fev[(sweep - 1) & 1]));
          const volatile int* fl = flag + 2 * ((sweep - 1) & 1);
          if (!fl[0]) {
            still_active = 0;
            break;
          }
          steps = std::min(steps, std::max(fl[1] - 1, 1));
        }
      }
      if (still_active && issued > 0) {
        HIPCHK(hipEventSynchronize(fev[(issued - 1) & 1]));
        still_active = flag[2 * ((issued - 1) & 1)];
      }
    }
    h->pool.push_back(fev[0]);
    h->pool.push_back(fev[1]);
    if (still_active && h->opts.max_sweeps > blocked) {
      Timer tp(h, K_JACOBI_AUX);
      STCHK(tp.start());
      HIPCHK(launch_jacobi_polish(d_secs, d_jlist, ns, scaled, d_acc, d_jst, h->opts.jacobi_tol,
                                  h->opts.max_sweeps - blocked, h->st));
      STCHK(tp.stop());
      h->stats.jacobi_aux_launches += 1;
      h->stats.polish_launches += 1;
    }
    Timer tf(h, K_JACOBI_AUX);
    STCHK(tf.start());
    HIPCHK(launch_jacobi_finalize(d_secs, d_jlist, ns, P.jmaxrows, scaled, d_acc, sig, ord, h->st));
    STCHK(tf.stop());
    h->stats.jacobi_aux_launches += 1;
  }
  {
    Timer tm(h, K_SELECT);
    STCHK(tm.start());
    HIPCHK(launch_select(d_gates, ng, d_secs, sig, static_cast<double*>(h->sel_v.p),
                         static_cast<int*>(h->sel_k.p), at<long long>(h->plan, o_seloff),
                         at<int>(h->plan, o_kept), at<CutOut>(h->plan, o_cut), P.maxP, sel_global, d_tbefore,
                         h->st));
    STCHK(tm.stop());
  }
  // read back kept counts, cut results and Jacobi statistics
  const size_t res_bytes = pk.total - o_kept;
  STCHK(ensure_pin(h->stage_res, res_bytes));
  HIPCHK(hipMemcpyAsync(h->stage_res.p, at<char>(h->plan, o_kept), res_bytes, hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  STCHK(drain_events(h));
  const char* rb = static_cast<const char*>(h->stage_res.p);
  const int* kept = reinterpret_cast<const int*>(rb);
  const CutOut* cut = reinterpret_cast<const CutOut*>(rb + (o_cut - o_kept));
  const JacobiOut* jst = reinterpret_cast<const JacobiOut*>(rb + (o_jst - o_kept));

  for (int s = 0; s < ns; ++s) {
    const SectorWork& sw = P.secs[s];
    if (!jst[s].converged)
      return fail(MPS_E_NOCONV, "Jacobi SVD of sector m=%d (%dx%d) did not converge in %d sweeps",
                  sw.m, sw.r, sw.c, h->opts.max_sweeps);
  }
  for (int g = 0; g < ng; ++g)
    if (cut[g].flags)
      return fail(MPS_E_NUMERIC, "two-site matrix at site %d vanished or is not finite", refs[g].site);
  for (int s = 0; s < ns; ++s) {
    mps_stats& gs = refs[P.secs[s].gate].h->stats;
    gs.sectors += 1;
    gs.sweeps += jst[s].sweeps;
    gs.rotations += jst[s].rotations;
    const double jf = 8.0 * double(jst[s].gram_units) + 8.0 * double(jst[s].apply_units);
    gs.jacobi_flops += jf;
    if (P.jblock == kJB8) gs.jacobi8_flops += jf;
  }
  h->stats.theta_flops += P.theta_flops;

  // new bond tables and update lists
  plan_t0 = clock::now();
  std::vector<RowWork> rows;
  std::vector<UpdateWork> upds(ng);
  std::vector<double2*> fill_ptr(ng);
  std::vector<long long> fill_cnt(ng);
  std::vector<std::vector<GemmWork>> gemms(1);   // per column block of the sectors
  long long maxfill = 0;
  std::vector<int> ntiles(1, 0);
  std::vector<Bond> newb(ng);
  for (int g = 0; g < ng; ++g) {
    mps_state* hg = refs[g].h;
    const int s = refs[g].site;
    const int chil = hg->bonds[s].dim();
    const int chir = hg->bonds[s + 2].dim();
    Bond& nb = newb[g];
    for (int i = P.gp[g].sec_begin; i < P.gp[g].sec_end; ++i) {
      if (kept[i] <= 0) continue;
      nb.charge.push_back(P.secs[i].m);
      nb.count.push_back(kept[i]);
    }
    nb.finish();
    const int chin = nb.dim();
    if (chin > hg->cap[s + 1] || chin <= 0)
      return fail(MPS_E_NUMERIC, "internal: new bond dimension %d outside 1..%d", chin, hg->cap[s + 1]);
    upds[g].br_new = hg->site[s + 1];
    upds[g].lam_new = hg->lam[s + 1];
    upds[g].ldr = chir;
    fill_ptr[g] = hg->site[s];
    fill_cnt[g] = (long long)chil * chin;
    maxfill = std::max(maxfill, fill_cnt[g]);
    int k = 0;
    for (int i = P.gp[g].sec_begin; i < P.gp[g].sec_end; ++i) {
      if (kept[i] <= 0) continue;
      const SectorWork& sw = P.secs[i];
      const int o = nb.off[k];
      for (int j = 0; j < kept[i]; ++j) rows.push_back({g, i, j, o + j});
      // new B[s](row block, kept) = sum over column blocks of
      // Theta~(row block, column block) V^dagger(kept, column block)^dagger,
      // column block kc in launch kc (accumulating after the first)
      for (int kc = 0; kc < sw.ncb; ++kc)
        for (int kr = 0; kr < sw.nrb; ++kr) {
          GemmWork gw{};
          gw.a = raw + sw.off + (size_t)sw.rb_pos[kr] * sw.c + sw.cb_pos[kc];
          gw.lda = sw.c;
          gw.b = hg->site[s + 1] + (size_t)o * chir + sw.cb_off[kc];
          gw.ldb = chir;
          gw.c = hg->site[s] + (size_t)sw.rb_off[kr] * chin + o;
          gw.ldc = chin;
          gw.m = sw.rb_n[kr];
          gw.n = kept[i];
          gw.k = sw.cb_n[kc];
          gw.opa = 0;
          gw.opb = 1;
          gw.beta_one = kc > 0 ? 1 : 0;
          gw.tiles_n = (gw.n + kGemmTile - 1) / kGemmTile;
          if ((int)gemms.size() <= kc) {
            gemms.resize(kc + 1);
            ntiles.resize(kc + 1, 0);
          }
          gw.tile_begin = ntiles[kc];
          ntiles[kc] += ((gw.m + kGemmTile - 1) / kGemmTile) * gw.tiles_n;
          gemms[kc].push_back(gw);
        }
      hg->stats.update_flops += 8.0 * sw.r * double(sw.c) * kept[i];
      ++k;
    }
  }
  Packer pu;
  const size_t u_rows = pu.add(rows.data(), rows.size() * sizeof(RowWork));
  const size_t u_upd = pu.add(upds.data(), upds.size() * sizeof(UpdateWork));
  const size_t u_fp = pu.add(fill_ptr.data(), fill_ptr.size() * sizeof(double2*));
  const size_t u_fc = pu.add(fill_cnt.data(), fill_cnt.size() * sizeof(long long));
  std::vector<size_t> u_gemm(gemms.size());
  for (size_t kc = 0; kc < gemms.size(); ++kc)
    u_gemm[kc] = pu.add(gemms[kc].data(), gemms[kc].size() * sizeof(GemmWork));
  STCHK(ensure(h, h->upd, pu.total));
  STCHK(ensure_pin(h->stage_upd, pu.total));
  pu.write(h->stage_upd.p);
  HIPCHK(hipMemcpyAsync(h->upd.p, h->stage_upd.p, pu.total, hipMemcpyHostToDevice, h->st));
  plan_add();
  {
    Timer tm(h, K_UPDATE);
    STCHK(tm.start());
    HIPCHK(launch_update_rows(at<RowWork>(h->upd, u_rows), (int)rows.size(), d_secs,
                              at<UpdateWork>(h->upd, u_upd), scaled, sig, ord, h->st));
    HIPCHK(launch_zero_fill(at<double2*>(h->upd, u_fp), at<long long>(h->upd, u_fc), ng, maxfill, h->st));
    for (size_t kc = 0; kc < gemms.size(); ++kc)
      HIPCHK(launch_zgemm(at<GemmWork>(h->upd, u_gemm[kc]), (int)gemms[kc].size(), ntiles[kc], h->st));
    STCHK(tm.stop());
  }
  for (int g = 0; g < ng; ++g)
    if (g == 0 || refs[g - 1].h != refs[g].h) refs[g].h->last_leak.clear();
  for (int g = 0; g < ng; ++g) {
    mps_state* hg = refs[g].h;
    hg->bonds[refs[g].site + 1] = newb[g];
    if (discarded) discarded[g] = cut[g].discarded;
    hg->last_leak.push_back(cut[g].leak);
    hg->stats.leak_total += cut[g].leak;
    hg->stats.gates += 1;
    hg->stats.max_discarded = std::max(hg->stats.max_discarded, cut[g].discarded);
    if (std::isfinite(cut[g].margin)) hg->stats.min_margin = std::min(hg->stats.min_margin, cut[g].margin);
    if (g == 0 || refs[g - 1].h != hg) hg->stats.layers += 1;
  }
  h->stats.theta_launches += 1;
  h->stats.select_launches += 1;
  h->stats.update_launches += 3;
  return MPS_OK;
}

// A dense gate may carry charge-changing elements up to this fraction of its
// largest element (rounding of a numerically built gate); they are dropped.
constexpr double kDenseLeak = 1e-13;

// Argument checks of one state's layer: sites in range, finite gates, disjoint
// pairs.  Gates are 2x2 mode unitaries, or with dense set d^2 x d^2 matrices
// that must conserve the local charge (p + q = a + b).
mps_status check_layer(mps_t h, int ngates, const int* sites, const mps_z* gs, bool dense = false) {
  if (!valid_handle(h)) return fail(MPS_E_ARG, "invalid handle");
  if (ngates < 0) return fail(MPS_E_ARG, "negative gate count");
  if (ngates == 0) return MPS_OK;
  if (!sites || !gs) return fail(MPS_E_ARG, "sites and gates are required");
  const int d = h->d, dd = d * d;
  const size_t gsz = dense ? (size_t)dd * dd : 4;
  if (!dense && !h->rule.photon)
    return fail(MPS_E_ARG, "only a U(1) photon-number state takes mode unitaries; use mps_apply_layer_dense");
  std::vector<int> order(ngates);
  for (int g = 0; g < ngates; ++g) {
    if (sites[g] < 0 || sites[g] > h->L - 2) return fail(MPS_E_ARG, "gate site %d outside 0..L-2", sites[g]);
    const mps_z* e = gs + gsz * g;
    double big = 0.0;
    for (size_t k = 0; k < gsz; ++k) {
      if (!std::isfinite(e[k].re) || !std::isfinite(e[k].im)) return fail(MPS_E_ARG, "non-finite gate element");
      big = std::max(big, std::hypot(e[k].re, e[k].im));
    }
    if (dense)
      for (int r = 0; r < dd; ++r)
        for (int c = 0; c < dd; ++c)
          if (!h->rule.conserves(r / d, r % d, c / d, c % d) &&
              std::hypot(e[r * dd + c].re, e[r * dd + c].im) > kDenseLeak * big)
            return fail(MPS_E_CHARGE, "gate %d: element (%d,%d) changes the local charge %d -> %d", g, r, c,
                        h->rule.step[c / d] + h->rule.step[c % d], h->rule.step[r / d] + h->rule.step[r % d]);
    order[g] = sites[g];
  }
  std::sort(order.begin(), order.end());
  for (int g = 1; g < ngates; ++g)
    if (order[g] - order[g - 1] < 2) return fail(MPS_E_ARG, "gates of one layer must act on disjoint site pairs");
  return MPS_OK;
}

mps_status destroy_buffers(mps_state* h) {
  if (h->st) (void)hipStreamSynchronize(h->st);
  if (h->cap_st) {
    (void)hipStreamDestroy(h->cap_st);
    h->cap_st = nullptr;
  }
  for (double* p : h->lam) dfree(h, p);
  for (double2* p : h->site) dfree(h, p);
  h->lam.clear();
  h->site.clear();
  DevBuf* bufs[] = {&h->th_raw, &h->th_scaled, &h->acc, &h->jperm, &h->jnorm, &h->sigma, &h->order, &h->plan, &h->upd,
                    &h->norm_e0, &h->norm_e1, &h->norm_t, &h->sel_v, &h->sel_k, &h->misc, &h->pbuf,
                    &h->planes, &h->envs, &h->samp, &h->tbefore};
  for (DevBuf* b : bufs) {
    dfree(h, b->p);
    b->p = nullptr;
    b->cap = 0;
  }
  PinBuf* pins[] = {&h->stage_plan, &h->stage_upd, &h->stage_res, &h->stage_misc, &h->stage_flag, &h->stage_samp};
  for (PinBuf* b : pins) {
    if (b->p) (void)hipHostFree(b->p);
    b->p = nullptr;
    b->cap = 0;
  }
  for (const Pending& p : h->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  h->pending.clear();
  for (hipEvent_t e : h->pool) (void)hipEventDestroy(e);
  h->pool.clear();
  return MPS_OK;
}

}  // namespace

// ============================================================================
extern "C" {

void mps_default_opts(mps_opts* o) {
  if (!o) return;
  o->chi_max = 0;
  o->cutoff = 0.0;
  o->zero_tol = 1e-13;
  o->max_sweeps = 40;
  o->jacobi_tol = 0.0;
  o->form = MPS_FORM_PLAIN_C128;
  o->modulus = 0;
  o->blocked_sweeps = 0;
  o->select_scratch = 0;
  o->sweep_graph = 0;
  o->tile_tuning = 1;
  o->jacobi_block = 0;
  o->jacobi_lockstep = 0;
}

const char* mps_last_error(void) { return g_err.c_str(); }

}  // extern "C"

namespace {

// mps_create for a given charge rule: `charges` of the rule's keys, n_photons
// the key of bond 0 (U(1) and Z_n: the photon number; the rule's steps then
// the identity).
mps_status create_impl(int L, int d, int n_photons, const int* bond_dim, const int* bond_charge,
                       const mps_z* const* gamma, const double* const* lambda, const mps_opts* opts,
                       const mps_device* dev, const std::vector<int>* steps, int ncomp, int radix,
                       mps_t* out) {
  if (!out) return fail(MPS_E_ARG, "out is NULL");
  *out = nullptr;
  if (L < 2) return fail(MPS_E_ARG, "L must be at least 2");
  if (d < 2 || d > kMaxD) return fail(MPS_E_ARG, "d must lie in 2..%d", kMaxD);
  if (n_photons < 0) return fail(MPS_E_ARG, "negative photon number");
  if (!bond_dim || !bond_charge) return fail(MPS_E_ARG, "bond_dim and bond_charge are required");
  if (gamma && !lambda) return fail(MPS_E_ARG, "lambda is required with gamma");
  if (bond_dim[0] != 1 || bond_dim[L] != 1) return fail(MPS_E_ARG, "bond 0 and bond L must have dimension 1");
  for (int b = 0; b <= L; ++b) {
    if (bond_dim[b] < 1) return fail(MPS_E_ARG, "bond %d has dimension %d", b, bond_dim[b]);
    if (!gamma && bond_dim[b] != 1) return fail(MPS_E_ARG, "a product state needs every bond of dimension 1");
  }
  mps_opts o;
  mps_default_opts(&o);
  if (opts) o = *opts;
  if (o.max_sweeps <= 0) return fail(MPS_E_ARG, "max_sweeps must be positive");
  if (o.blocked_sweeps < 0) return fail(MPS_E_ARG, "blocked_sweeps must be >= 0");
  if (o.select_scratch != 0 && o.select_scratch != 1) return fail(MPS_E_ARG, "select_scratch must be 0 or 1");
  if (o.sweep_graph != 0 && o.sweep_graph != 1) return fail(MPS_E_ARG, "sweep_graph must be 0 or 1");
  if (o.tile_tuning < 0 || o.tile_tuning > 1 + kSgVariants)
    return fail(MPS_E_ARG, "tile_tuning must lie in 0..%d", 1 + kSgVariants);
  if (o.jacobi_block != 0 && o.jacobi_block != kJB8 && o.jacobi_block != kJB)
    return fail(MPS_E_ARG, "jacobi_block must be 0, %d or %d", kJB8, kJB);
  if (o.jacobi_lockstep != 0 && o.jacobi_lockstep != 1) return fail(MPS_E_ARG, "jacobi_lockstep must be 0 or 1");
  if (!(o.cutoff >= 0.0) || !(o.zero_tol >= 0.0)) return fail(MPS_E_ARG, "cutoff and zero_tol must be >= 0");
  if (o.form != MPS_FORM_PLAIN_C128 && o.form != MPS_FORM_SPLIT_BF16X3) return fail(MPS_E_ARG, "unknown form %d", o.form);
  // a Z_n charge gives each local occupation its own charge: n >= d
  if (o.modulus != 0 && (o.modulus < 2 || o.modulus < d))
    return fail(MPS_E_ARG, "a Z_n charge needs n >= 2 and n at least the local dimension (modulus %d, d %d)",
                o.modulus, d);
  const int zn = o.modulus;
  const int nq = zn ? n_photons % zn : n_photons;     // charge of bond 0
  ChargeRule R;
  {
    std::vector<int> ident(d);
    for (int p = 0; p < d; ++p) ident[p] = p;
    if (steps && zn) return fail(MPS_E_ARG, "a Z_n charge takes the occupations as its charges");
    R.init(zn, steps ? *steps : ident);
  }

  // charge tables with a stable sort of every bond by charge
  std::vector<Bond> bonds(L + 1);
  std::vector<std::vector<int>> perm(L + 1);
  size_t pos = 0;
  for (int b = 0; b <= L; ++b) {
    const int n = bond_dim[b];
    std::vector<int> ch(bond_charge + pos, bond_charge + pos + n);
    pos += n;
    for (int c : ch)
      if (c < 0 || c > (zn ? zn - 1 : n_photons))
        return fail(MPS_E_CHARGE, "bond %d has charge %d outside 0..%d", b, c, zn ? zn - 1 : n_photons);
    std::vector<int> idx(n);
    for (int i = 0; i < n; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int c) { return ch[a] < ch[c]; });
    perm[b] = idx;
    Bond& B = bonds[b];
    for (int i = 0; i < n; ++i) {
      const int c = ch[idx[i]];
      if (B.charge.empty() || B.charge.back() != c) {
        B.charge.push_back(c);
        B.count.push_back(0);
      }
      B.count.back() += 1;
    }
    B.finish();
  }
  if (bonds[0].charge[0] != nq) return fail(MPS_E_CHARGE, "bond 0 must carry charge N (Eq. E4)");
  if (bonds[L].charge[0] != 0) return fail(MPS_E_CHARGE, "bond L must carry charge 0 (Eq. E4)");
  // every left charge must connect to some right charge with 0 <= cL - cR <= d-1
  for (int s = 0; s < L; ++s) {
    for (int c : bonds[s].charge) {
      bool ok = false;
      for (int c2 : bonds[s + 1].charge)
        if (R.ok(c, c2)) ok = true;
      if (!ok) return fail(MPS_E_CHARGE, "charge %d on bond %d has no admissible partner on bond %d", c, s, s + 1);
    }
  }
  // host site tensors B = Gamma * lambda_{s+1}, in sorted order, checked against Eq. (E2)
  std::vector<std::vector<double2>> hsite(L);
  std::vector<std::vector<double>> hlam(L + 1);
  pos = 0;
  std::vector<size_t> start(L + 1);
  for (int b = 0; b <= L; ++b) {
    start[b] = pos;
    pos += bond_dim[b];
  }
  for (int b = 0; b <= L; ++b) {
    hlam[b].resize(bond_dim[b]);
    for (int i = 0; i < bond_dim[b]; ++i) {
      const double v = lambda ? lambda[b][perm[b][i]] : 1.0;
      if (!std::isfinite(v)) return fail(MPS_E_ARG, "non-finite lambda on bond %d", b);
      hlam[b][i] = v;
    }
  }
  for (int s = 0; s < L; ++s) {
    const int rdim = bond_dim[s], cdim = bond_dim[s + 1];
    hsite[s].assign((size_t)rdim * cdim, make_double2(0.0, 0.0));
    for (int i = 0; i < rdim; ++i) {
      const int ci = bond_charge[start[s] + perm[s][i]];
      for (int j = 0; j < cdim; ++j) {
        const int cj = bond_charge[start[s + 1] + perm[s + 1][j]];
        double2 v;
        if (gamma) {
          const mps_z z = gamma[s][(size_t)perm[s][i] * cdim + perm[s + 1][j]];
          v = make_double2(z.re * hlam[s + 1][j], z.im * hlam[s + 1][j]);
          const bool allowed = R.ok(ci, cj);
          if (!allowed && (z.re != 0.0 || z.im != 0.0))
            return fail(MPS_E_CHARGE, "site %d entry (%d,%d) violates the charge rule (Eq. E2)", s, i, j);
          if (!std::isfinite(z.re) || !std::isfinite(z.im)) return fail(MPS_E_ARG, "non-finite gamma");
        } else {
          v = R.ok(ci, cj) ? make_double2(1.0, 0.0) : make_double2(0.0, 0.0);
        }
        hsite[s][(size_t)i * cdim + j] = v;
      }
    }
  }

  mps_state* h = new (std::nothrow) mps_state();
  if (!h) return fail(MPS_E_NOMEM, "handle allocation failed");
  h->L = L;
  h->d = d;
  h->N = nq;
  h->mod = zn;
  h->rule = R;
  h->ncomp = ncomp;
  h->radix = radix;
  h->opts = o;
  if (dev) h->dev = *dev;
  h->st = static_cast<hipStream_t>(h->dev.stream);
  if (hipGetDevice(&h->device) != hipSuccess) h->device = 0;
  if (hipDeviceGetAttribute(&h->cus, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess || h->cus < 1)
    h->cus = 256;
  h->bonds = bonds;
  h->stats.min_margin = INFINITY;
  mps_status s = compute_caps(h);
  if (s != MPS_OK) {
    delete h;
    return s;
  }
  h->lam.assign(L + 1, nullptr);
  h->site.assign(L, nullptr);
  for (int b = 0; b <= L && s == MPS_OK; ++b) {
    h->lam[b] = static_cast<double*>(dalloc(h, (size_t)h->cap[b] * sizeof(double)));
    if (!h->lam[b]) s = fail(MPS_E_NOMEM, "lambda allocation failed");
  }
  for (int t = 0; t < L && s == MPS_OK; ++t) {
    h->site[t] = static_cast<double2*>(dalloc(h, (size_t)h->cap[t] * h->cap[t + 1] * sizeof(double2)));
    if (!h->site[t]) s = fail(MPS_E_NOMEM, "site allocation failed");
  }
  if (s == MPS_OK) {
    // upload through pinned staging, one synchronisation
    size_t bytes = 0;
    for (int b = 0; b <= L; ++b) bytes = align256(bytes + hlam[b].size() * sizeof(double));
    for (int t = 0; t < L; ++t) bytes = align256(bytes + hsite[t].size() * sizeof(double2));
    s = ensure_pin(h->stage_misc, bytes);
    if (s == MPS_OK) {
      char* base = static_cast<char*>(h->stage_misc.p);
      size_t o2 = 0;
      hipError_t e = hipSuccess;
      for (int b = 0; b <= L && e == hipSuccess; ++b) {
        const size_t nb = hlam[b].size() * sizeof(double);
        std::memcpy(base + o2, hlam[b].data(), nb);
        e = hipMemcpyAsync(h->lam[b], base + o2, nb, hipMemcpyHostToDevice, h->st);
        o2 = align256(o2 + nb);
      }
      for (int t = 0; t < L && e == hipSuccess; ++t) {
        const size_t nb = hsite[t].size() * sizeof(double2);
        std::memcpy(base + o2, hsite[t].data(), nb);
        e = hipMemcpyAsync(h->site[t], base + o2, nb, hipMemcpyHostToDevice, h->st);
        o2 = align256(o2 + nb);
      }
      if (e == hipSuccess) e = hipStreamSynchronize(h->st);
      if (e != hipSuccess) s = fail(MPS_E_DEVICE, "upload failed: %s", hipGetErrorString(e));
    }
  }
  if (s != MPS_OK) {
    destroy_buffers(h);
    delete h;
    return s;
  }
  *out = h;
  return MPS_OK;
}

}  // namespace

extern "C" {

mps_status mps_create(int L, int d, int n_photons, const int* bond_dim, const int* bond_charge,
                      const mps_z* const* gamma, const double* const* lambda, const mps_opts* opts,
                      const mps_device* dev, mps_t* out) {
  return create_impl(L, d, n_photons, bond_dim, bond_charge, gamma, lambda, opts, dev, nullptr, 1, 0, out);
}

mps_status mps_create_product_charges(int L, int d, const int* occupation, int ncomp, const int* charge_map,
                                      const mps_opts* opts, const mps_device* dev, mps_t* out) {
  if (!out) return fail(MPS_E_ARG, "out is NULL");
  *out = nullptr;
  if (!occupation || !charge_map) return fail(MPS_E_ARG, "occupation and charge_map are required");
  if (L < 2) return fail(MPS_E_ARG, "L must be at least 2");
  if (d < 2 || d > kMaxD) return fail(MPS_E_ARG, "d must lie in 2..%d", kMaxD);
  if (ncomp != 1 && ncomp != 2) return fail(MPS_E_ARG, "ncomp must be 1 or 2");
  if (opts && opts->modulus != 0) return fail(MPS_E_ARG, "charge_map takes U(1) components (modulus 0)");
  for (int i = 0; i < L; ++i)
    if (occupation[i] < 0 || occupation[i] >= d)
      return fail(MPS_E_ARG, "local state %d of mode %d outside 0..d-1", occupation[i], i);
  std::vector<long long> tot(ncomp, 0), mx(ncomp, 0);
  for (int p = 0; p < d; ++p)
    for (int k = 0; k < ncomp; ++k) {
      const int v = charge_map[p * ncomp + k];
      if (v < 0 || v > 64) return fail(MPS_E_ARG, "charge_map entry %d outside 0..64", v);
      mx[k] = std::max<long long>(mx[k], v);
    }
  for (int i = 0; i < L; ++i)
    for (int k = 0; k < ncomp; ++k) tot[k] += charge_map[occupation[i] * ncomp + k];
  // keys: radix above twice the second components a bond difference or a
  // two-site total can carry
  const long long radix = ncomp == 2 ? 2 * (tot[1] + mx[1]) + 2 : 0;
  if (ncomp == 2 && (tot[0] + 1) * radix > (1LL << 24)) return fail(MPS_E_ARG, "charges too large to pack");
  std::vector<int> steps(d);
  for (int p = 0; p < d; ++p)
    steps[p] = ncomp == 2 ? int(charge_map[2 * p] * radix + charge_map[2 * p + 1]) : charge_map[p];
  for (int p = 0; p < d; ++p)
    for (int q = 0; q < p; ++q)
      if (steps[p] == steps[q]) return fail(MPS_E_ARG, "local states %d and %d carry the same charge", q, p);
  std::vector<int> dims(L + 1, 1), ch(L + 1, 0);
  long long c = 0;
  for (int i = 0; i < L; ++i) c += steps[occupation[i]];
  const int total = int(c);
  for (int b = 0; b <= L; ++b) {
    ch[b] = int(c);
    if (b < L) c -= steps[occupation[b]];
  }
  return create_impl(L, d, total, dims.data(), ch.data(), nullptr, nullptr, opts, dev, &steps, ncomp, int(radix),
                     out);
}

mps_status mps_bond_charges(mps_t h, int bond, int cap, int* nsec, int* comps, int* count) {
  if (!valid_handle(h)) return fail(MPS_E_ARG, "invalid handle");
  if (bond < 0 || bond > h->L) return fail(MPS_E_ARG, "bond %d outside 0..L", bond);
  const Bond& B = h->bonds[bond];
  if (nsec) *nsec = (int)B.charge.size();
  if ((int)B.charge.size() > cap) return fail(MPS_E_ARG, "capacity %d < %zu sectors", cap, B.charge.size());
  for (size_t i = 0; i < B.charge.size(); ++i) {
    if (comps) {
      if (h->ncomp == 2) {
        comps[2 * i] = B.charge[i] / h->radix;
        comps[2 * i + 1] = B.charge[i] % h->radix;
      } else {
        comps[i] = B.charge[i];
      }
    }
    if (count) count[i] = B.count[i];
  }
  return MPS_OK;
}

mps_status mps_charge_components(mps_t h, int* ncomp) {
  if (!valid_handle(h)) return fail(MPS_E_ARG, "invalid handle");
  if (!ncomp) return fail(MPS_E_ARG, "ncomp is NULL");
  *ncomp = h->ncomp;
  return MPS_OK;
}

mps_status mps_create_product(int L, int d, const int* occupation, const mps_opts* opts,
                              const mps_device* dev, mps_t* out) {
  if (!occupation) return fail(MPS_E_ARG, "occupation is NULL");
  if (L < 2) return fail(MPS_E_ARG, "L must be at least 2");
  std::vector<int> dims(L + 1, 1), ch(L + 1, 0);
  int N = 0;
  for (int i = 0; i < L; ++i) {
    if (occupation[i] < 0 || occupation[i] >= d)
      return fail(MPS_E_ARG, "occupation %d of mode %d outside 0..d-1", occupation[i], i);
    N += occupation[i];
  }
  const int zn = opts ? opts->modulus : 0;
  int c = N;
  for (int b = 0; b <= L; ++b) {
    ch[b] = (zn > 0) ? c % zn : c;
    if (b < L) c -= occupation[b];
  }
  return mps_create(L, d, N, dims.data(), ch.data(), nullptr, nullptr, opts, dev, out);
}

mps_status mps_destroy(mps_t h) {
  if (!h) return MPS_OK;
  destroy_buffers(h);
  delete h;
  return MPS_OK;
}

mps_status mps_apply_layer(mps_t h, int ngates, const int* sites, const mps_z* u2s, double* discarded) {
  STCHK(check_layer(h, ngates, sites, u2s));
  if (ngates == 0) return MPS_OK;
  std::vector<GateRef> refs(ngates);
  for (int g = 0; g < ngates; ++g) refs[g] = {h, sites[g], u2s + 4 * g, nullptr};
  return apply_batch(refs, discarded);
}

mps_status mps_apply_layer_dense(mps_t h, int ngates, const int* sites, const mps_z* g4s, double* discarded) {
  STCHK(check_layer(h, ngates, sites, g4s, true));
  if (ngates == 0) return MPS_OK;
  const size_t gsz = (size_t)h->d * h->d * h->d * h->d;
  std::vector<GateRef> refs(ngates);
  for (int g = 0; g < ngates; ++g) refs[g] = {h, sites[g], nullptr, g4s + gsz * g};
  return apply_batch(refs, discarded);
}

mps_status mps_apply_batch(int nh, const mps_t* hs, const int* ngates, const int* sites, const mps_z* u2s,
                           double* discarded) {
  if (nh < 0) return fail(MPS_E_ARG, "negative state count");
  if (nh == 0) return MPS_OK;
  if (!hs || !ngates) return fail(MPS_E_ARG, "hs and ngates are required");
  std::vector<GateRef> refs;
  long long off = 0;
  for (int i = 0; i < nh; ++i) {
    mps_t h = hs[i];
    if (!valid_handle(h)) return fail(MPS_E_ARG, "invalid handle at index %d", i);
    for (int k = 0; k < i; ++k)
      if (hs[k] == h) return fail(MPS_E_ARG, "state %d appears twice in one batch", i);
    if (ngates[i] < 0) return fail(MPS_E_ARG, "negative gate count for state %d", i);
    if (ngates[i] == 0) continue;
    if (!sites || !u2s) return fail(MPS_E_ARG, "sites and u2s are required");
    STCHK(check_layer(h, ngates[i], sites + off, u2s + 4 * off));
    if (!refs.empty()) {
      mps_state* h0 = refs[0].h;
      if (h->d != h0->d) return fail(MPS_E_ARG, "states of one batch must share the local dimension");
      if (h->st != h0->st) return fail(MPS_E_ARG, "states of one batch must share one stream");
      if (h->opts.form != h0->opts.form) return fail(MPS_E_ARG, "states of one batch must share the form");
    }
    for (int g = 0; g < ngates[i]; ++g) refs.push_back({h, sites[off + g], u2s + 4 * (off + g), nullptr});
    off += ngates[i];
  }
  if (refs.empty()) return MPS_OK;
  return apply_batch(refs, discarded);
}

mps_status mps_apply_gate(mps_t h, int site, const mps_z u2[4], double* discarded) {
  if (!u2) return fail(MPS_E_ARG, "u2 is NULL");
  return mps_apply_layer(h, 1, &site, u2, discarded);
}

mps_status mps_truncate(mps_t h, int bond, int chi_max, double cutoff, double* discarded) {
  if (!valid_handle(h)) return fail(MPS_E_ARG, "invalid handle");
  if (bond < 1 || bond > h->L - 1) return fail(MPS_E_ARG, "bond %d outside 1..L-1", bond);
  if (!(cutoff >= 0.0)) return fail(MPS_E_ARG, "cutoff must be >= 0");
  const Bond& B = h->bonds[bond];
  std::vector<SectorWork> secs(B.charge.size());
  int T = 0;
  for (size_t i = 0; i < B.charge.size(); ++i) {
    SectorWork sw{};
    sw.gate = 0;
    sw.m = B.charge[i];
    sw.r = B.count[i];
    sw.c = B.count[i];
    sw.sig = B.off[i];
    sw.kmax = B.count[i];
    secs[i] = sw;
    T += sw.kmax;
  }
  GateWork gw{};
  gw.sec_begin = 0;
  gw.sec_end = (int)secs.size();
  gw.keep_cap = h->cap[bond];
  gw.chi_max = chi_max;
  gw.cutoff = cutoff;
  gw.zero_tol = h->opts.zero_tol;
  if (secs.size() > 1024) return fail(MPS_E_ARG, "more than 1024 charges on bond %d", bond);
  int Pp = 1;
  while (Pp < T) Pp <<= 1;
  const bool sel_global = Pp > kSelectLds || h->opts.select_scratch;
  long long zero = 0;
  Packer pk;
  const size_t o_g = pk.add(&gw, sizeof gw);
  const size_t o_s = pk.add(secs.data(), secs.size() * sizeof(SectorWork));
  const size_t o_z = pk.add(&zero, sizeof zero);
  const size_t o_kept = pk.add(nullptr, secs.size() * sizeof(int));
  const size_t o_cut = pk.add(nullptr, sizeof(CutOut));
  STCHK(ensure(h, h->plan, pk.total));
  STCHK(ensure_pin(h->stage_plan, pk.total));
  if (sel_global) {
    STCHK(ensure(h, h->sel_v, (size_t)Pp * sizeof(double)));
    STCHK(ensure(h, h->sel_k, (size_t)Pp * sizeof(int)));
  }
  HIPCHK(hipStreamSynchronize(h->st));
  pk.write(h->stage_plan.p);
  HIPCHK(hipMemcpyAsync(h->plan.p, h->stage_plan.p, o_kept, hipMemcpyHostToDevice, h->st));
  HIPCHK(launch_select(at<GateWork>(h->plan, o_g), 1, at<SectorWork>(h->plan, o_s), h->lam[bond],
                       static_cast<double*>(h->sel_v.p), static_cast<int*>(h->sel_k.p),
                       at<long long>(h->plan, o_z), at<int>(h->plan, o_kept), at<CutOut>(h->plan, o_cut),
                       Pp, sel_global, nullptr, h->st));
  STCHK(ensure_pin(h->stage_res, pk.total - o_kept));
  HIPCHK(hipMemcpyAsync(h->stage_res.p, at<char>(h->plan, o_kept), pk.total - o_kept,
                        hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  const int* kept = static_cast<const int*>(h->stage_res.p);
  CutOut co;
  std::memcpy(&co, static_cast<const char*>(h->stage_res.p) + (o_cut - o_kept), sizeof co);
  if (co.flags) return fail(MPS_E_NUMERIC, "bond %d has no positive finite Schmidt value", bond);
  // maps of kept indices (each charge keeps its leading values)
  Bond nb;
  std::vector<int> map;
  for (size_t i = 0; i < secs.size(); ++i) {
    if (kept[i] <= 0) continue;
    nb.charge.push_back(B.charge[i]);
    nb.count.push_back(kept[i]);
    for (int j = 0; j < kept[i]; ++j) map.push_back(B.off[i] + j);
  }
  nb.finish();
  const int chin = nb.dim();
  const int chil = h->bonds[bond - 1].dim(), chio = B.dim(), chir = h->bonds[bond + 1].dim();
  const size_t tmp_elems = std::max((size_t)chil * chin, (size_t)chin * chir) + (size_t)chin;
  STCHK(ensure(h, h->misc, align256(map.size() * sizeof(int)) + tmp_elems * sizeof(double2)));
  STCHK(ensure_pin(h->stage_misc, map.size() * sizeof(int)));
  std::memcpy(h->stage_misc.p, map.data(), map.size() * sizeof(int));
  int* d_map = static_cast<int*>(h->misc.p);
  double2* tmp = at<double2>(h->misc, align256(map.size() * sizeof(int)));
  HIPCHK(hipMemcpyAsync(d_map, h->stage_misc.p, map.size() * sizeof(int), hipMemcpyHostToDevice, h->st));
  HIPCHK(launch_gather_cols(h->site[bond - 1], chio, tmp, chin, chil, d_map, chin, h->st));
  HIPCHK(hipMemcpyAsync(h->site[bond - 1], tmp, (size_t)chil * chin * sizeof(double2), hipMemcpyDeviceToDevice, h->st));
  HIPCHK(launch_gather_rows(h->site[bond], chir, tmp, chir, d_map, chin, chir, h->st));
  HIPCHK(hipMemcpyAsync(h->site[bond], tmp, (size_t)chin * chir * sizeof(double2), hipMemcpyDeviceToDevice, h->st));
  double* tl = reinterpret_cast<double*>(tmp);
  HIPCHK(launch_gather_vec(h->lam[bond], tl, d_map, chin, h->st));
  HIPCHK(hipMemcpyAsync(h->lam[bond], tl, (size_t)chin * sizeof(double), hipMemcpyDeviceToDevice, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  h->bonds[bond] = nb;
  if (discarded) *discarded = co.discarded;
  return MPS_OK;
}

mps_status mps_amplitude(mps_t h, int count, const int* occ, mps_z* out) {
  if (!valid_handle(h)) return fail(MPS_E_ARG, "invalid handle");
  if (count < 0) return fail(MPS_E_ARG, "negative count");
  if (count == 0) return MPS_OK;
  if (!occ || !out) return fail(MPS_E_ARG, "occ and out are required");
  const int L = h->L, N = h->N;
  const int ncb = h->mod ? h->mod : N + 1;          // bondmap entries per bond
  std::vector<int2> bmap((size_t)(L + 1) * ncb, make_int2(0, 0));
  int maxdim = 1;
  for (int b = 0; b <= L; ++b) {
    const Bond& B = h->bonds[b];
    for (size_t i = 0; i < B.charge.size(); ++i)
      bmap[(size_t)b * ncb + B.charge[i]] = make_int2(B.off[i], B.count[i]);
    maxdim = std::max(maxdim, B.dim());
  }
  std::vector<int> ld(L);
  std::vector<const double2*> sp(L);
  for (int s = 0; s < L; ++s) {
    ld[s] = h->bonds[s + 1].dim();
    sp[s] = h->site[s];
  }
  Packer pk;
  const size_t o_sp = pk.add(sp.data(), sp.size() * sizeof(double2*));
  const size_t o_ld = pk.add(ld.data(), ld.size() * sizeof(int));
  const size_t o_bm = pk.add(bmap.data(), bmap.size() * sizeof(int2));
  const size_t o_occ = pk.add(occ, (size_t)count * L * sizeof(int));
  const size_t o_out = pk.add(nullptr, (size_t)count * sizeof(double2));
  if ((size_t)2 * maxdim * sizeof(double2) > 64 * 1024) return fail(MPS_E_ARG, "bond dimension too large for the amplitude kernel");
  STCHK(ensure(h, h->misc, pk.total));
  HIPCHK(hipStreamSynchronize(h->st));
  STCHK(ensure_pin(h->stage_misc, pk.total));
  pk.write(h->stage_misc.p);
  HIPCHK(hipMemcpyAsync(h->misc.p, h->stage_misc.p, o_out, hipMemcpyHostToDevice, h->st));
  HIPCHK(launch_amplitude(at<const double2*>(h->misc, o_sp), at<int>(h->misc, o_ld), at<int2>(h->misc, o_bm),
                          at<int>(h->misc, o_occ), at<double2>(h->misc, o_out), count, L, h->d, N, h->mod,
                          maxdim, steps_of(h), h->st));
  HIPCHK(hipMemcpyAsync(static_cast<char*>(h->stage_misc.p) + o_out, at<char>(h->misc, o_out),
                        (size_t)count * sizeof(double2), hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  std::memcpy(out, static_cast<char*>(h->stage_misc.p) + o_out, (size_t)count * sizeof(double2));
  return MPS_OK;
}

// Left environments E_0 .. E_L into the frames eb[b] (dim_b x dim_b, row-major):
// E_0 = 1 and E_{s+1}[c', c'] = sum_w B[w, c']^dagger E_s[w, w] B[w, c'], w the
// rows of bond s whose charges c' .. c'+d-1 reach charge c' of bond s+1, so
// every E is block-diagonal by charge.  eb[s] and eb[s+2] may be one frame.
//
// Work lists of the left-environment contraction (the norm's and the
// sampler's): per site s, T_c' = E_s[w, w] B[s][w, c'] into tbuf, then
// E_{s+1}[c', c'] = B[s][w, c']^dagger T_c', block by block over the charges
// c' of bond s+1 (w: the rows of bond s that reach c').  The packed lists stay
// valid while the EnvPlan lives (the packer keeps pointers into it).
struct EnvPlan {
  std::vector<std::vector<GemmWork>> p1, p2;
  std::vector<int> nt1, nt2;
  std::vector<double2*> fptr;
  std::vector<long long> fcnt;
  std::vector<size_t> o1, o2;
  size_t o_fp = 0, o_fc = 0, o_one = 0;
  double2 one = make_double2(1.0, 0.0);
  Packer pk;
  EnvPlan() = default;
  EnvPlan(const EnvPlan&) = delete;
  EnvPlan& operator=(const EnvPlan&) = delete;
};

// The largest bond dimension of the state and T's size in elements (d * that^2).
size_t env_tbuf_elems(const mps_state* h, int* maxdim_out) {
  int maxdim = 1;
  for (int b = 0; b <= h->L; ++b) maxdim = std::max(maxdim, h->bonds[b].dim());
  if (maxdim_out) *maxdim_out = maxdim;
  return (size_t)h->d * maxdim * maxdim;
}

mps_status plan_envs(mps_state* h, const std::vector<double2*>& eb, double2* tbuf, size_t tcap, EnvPlan& E) {
  const int L = h->L;
  E.p1.assign(L, {});
  E.p2.assign(L, {});
  E.nt1.assign(L, 0);
  E.nt2.assign(L, 0);
  E.fptr.assign(L, nullptr);
  E.fcnt.assign(L, 0);
  for (int s = 0; s < L; ++s) {
    const Bond& B0 = h->bonds[s];
    const Bond& B1 = h->bonds[s + 1];
    const int ld0 = B0.dim(), ld1 = B1.dim();
    double2* ein = eb[s];
    double2* eout = eb[s + 1];
    E.fptr[s] = eout;
    E.fcnt[s] = (long long)ld1 * ld1;
    size_t toff = 0;
    for (size_t i = 0; i < B1.charge.size(); ++i) {
      const int cp = B1.charge[i];
      // rows of bond s reaching charge cp: charges cp + step[p] (Z_n: taken
      // as all).  The range from the smallest to the largest such charge may hold
      // other charges too; their entries of B[s] are structural zeros, so they
      // add nothing (U(1): exactly the charges cp..cp+d-1)
      const int w0 = h->mod ? 0 : B0.off[B0.lower(cp + h->rule.minstep)];
      const int w1 = h->mod ? B0.dim() : B0.off[B0.lower(cp + h->rule.maxstep + 1)];
      if (w1 <= w0) continue;
      const int nn = B1.count[i], o1 = B1.off[i], kw = w1 - w0;
      GemmWork a{};
      a.a = ein + (size_t)w0 * ld0 + w0;
      a.lda = ld0;
      a.b = h->site[s] + (size_t)w0 * ld1 + o1;
      a.ldb = ld1;
      a.c = tbuf + toff;
      a.ldc = nn;
      a.m = kw;
      a.n = nn;
      a.k = kw;
      a.tiles_n = (nn + kGemmTile - 1) / kGemmTile;
      a.tile_begin = E.nt1[s];
      E.nt1[s] += ((kw + kGemmTile - 1) / kGemmTile) * a.tiles_n;
      E.p1[s].push_back(a);
      GemmWork b{};
      b.a = h->site[s] + (size_t)w0 * ld1 + o1;
      b.lda = ld1;
      b.opa = 1;
      b.b = tbuf + toff;
      b.ldb = nn;
      b.c = eout + (size_t)o1 * ld1 + o1;
      b.ldc = ld1;
      b.m = nn;
      b.n = nn;
      b.k = kw;
      b.tiles_n = (nn + kGemmTile - 1) / kGemmTile;
      b.tile_begin = E.nt2[s];
      E.nt2[s] += ((nn + kGemmTile - 1) / kGemmTile) * b.tiles_n;
      E.p2[s].push_back(b);
      toff += (size_t)kw * nn;
    }
    if (toff > tcap) return fail(MPS_E_ARG, "internal: environment scratch too small");
  }
  E.o1.assign(L, 0);
  E.o2.assign(L, 0);
  for (int s = 0; s < L; ++s) {
    E.o1[s] = E.pk.add(E.p1[s].data(), E.p1[s].size() * sizeof(GemmWork));
    E.o2[s] = E.pk.add(E.p2[s].data(), E.p2[s].size() * sizeof(GemmWork));
  }
  E.o_fp = E.pk.add(E.fptr.data(), E.fptr.size() * sizeof(double2*));
  E.o_fc = E.pk.add(E.fcnt.data(), E.fcnt.size() * sizeof(long long));
  E.o_one = E.pk.add(&E.one, sizeof E.one);
  return MPS_OK;
}

// The contraction's launches, with the packed lists already at `list` on the
// device: E_0 = 1, then per site a zero fill of E_{s+1} and the two products.
mps_status launch_envs(mps_state* h, const std::vector<double2*>& eb, const EnvPlan& E, char* list) {
  auto on = [&](size_t off) { return list + off; };
  HIPCHK(hipMemcpyAsync(eb[0], on(E.o_one), sizeof(double2), hipMemcpyDeviceToDevice, h->st));
  for (int s = 0; s < h->L; ++s) {
    HIPCHK(launch_zero_fill(reinterpret_cast<double2**>(on(E.o_fp)) + s,
                            reinterpret_cast<long long*>(on(E.o_fc)) + s, 1, E.fcnt[s], h->st));
    HIPCHK(launch_zgemm(reinterpret_cast<const GemmWork*>(on(E.o1[s])), (int)E.p1[s].size(), E.nt1[s], h->st));
    HIPCHK(launch_zgemm(reinterpret_cast<const GemmWork*>(on(E.o2[s])), (int)E.p2[s].size(), E.nt2[s], h->st));
  }
  return MPS_OK;
}

// The environments E_0..E_L into eb (device buffers of dim_b^2), through the
// handle's workspaces (misc, stage_misc); `extra` bytes of pinned staging are
// reserved after the uploaded lists, at offset *tail of stage_misc, for the
// caller.
mps_status left_envs(mps_state* h, const std::vector<double2*>& eb, size_t extra, size_t* tail) {
  const size_t tel = env_tbuf_elems(h, nullptr);
  STCHK(ensure(h, h->norm_t, tel * sizeof(double2)));
  EnvPlan E;
  STCHK(plan_envs(h, eb, static_cast<double2*>(h->norm_t.p), tel, E));
  HIPCHK(hipStreamSynchronize(h->st));
  STCHK(ensure(h, h->misc, E.pk.total));
  STCHK(ensure_pin(h->stage_misc, E.pk.total + extra));
  E.pk.write(h->stage_misc.p);
  HIPCHK(hipMemcpyAsync(h->misc.p, h->stage_misc.p, E.pk.total, hipMemcpyHostToDevice, h->st));
  STCHK(launch_envs(h, eb, E, static_cast<char*>(h->misc.p)));
  *tail = E.pk.total;
  return MPS_OK;
}

mps_status mps_norm(mps_t h, double* norm2) {
  if (!valid_handle(h)) return fail(MPS_E_ARG, "invalid handle");
  if (!norm2) return fail(MPS_E_ARG, "norm2 is NULL");
  const int L = h->L;
  int maxdim = 1;
  for (int b = 0; b <= L; ++b) maxdim = std::max(maxdim, h->bonds[b].dim());
  const size_t esz = (size_t)maxdim * maxdim;
  STCHK(ensure(h, h->norm_e0, esz * sizeof(double2)));
  STCHK(ensure(h, h->norm_e1, esz * sizeof(double2)));
  std::vector<double2*> eb(L + 1);
  for (int b = 0; b <= L; ++b)
    eb[b] = static_cast<double2*>((b & 1) ? h->norm_e1.p : h->norm_e0.p);
  size_t tail = 0;
  STCHK(left_envs(h, eb, sizeof(double2), &tail));
  double2* res = reinterpret_cast<double2*>(static_cast<char*>(h->stage_misc.p) + tail);
  HIPCHK(hipMemcpyAsync(res, eb[L], sizeof(double2), hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  *norm2 = res->x;
  return MPS_OK;
}

mps_status mps_norm_noalloc(mps_t h, double* norm2) {
  if (!valid_handle(h)) return fail(MPS_E_ARG, "invalid handle");
  if (!norm2) return fail(MPS_E_ARG, "norm2 is NULL");
  const int L = h->L;
  int maxdim = 1;
  const size_t tel = env_tbuf_elems(h, &maxdim);
  const size_t esz = (size_t)maxdim * maxdim;
  // scratch layout: E (even bonds) | E (odd bonds) | T | packed work lists
  const size_t o_e1 = align256(esz * sizeof(double2));
  const size_t o_t = o_e1 + align256(esz * sizeof(double2));
  const size_t o_list = o_t + align256(tel * sizeof(double2));
  int cur = 0;
  HIPCHK(hipGetDevice(&cur));
  struct DeviceGuard {
    int prev, want;
    ~DeviceGuard() {
      if (prev != want) (void)hipSetDevice(prev);
    }
  } guard{cur, h->device};
  if (cur != h->device) HIPCHK(hipSetDevice(h->device));
  auto lock = scratch_lock();
  void* base = nullptr;
  size_t cap = 0;
  HIPCHK(scratch_region(h->device, &base, &cap));
  char* sc = static_cast<char*>(base);
  std::vector<double2*> eb(L + 1);
  for (int b = 0; b <= L; ++b) eb[b] = reinterpret_cast<double2*>(sc + ((b & 1) ? o_e1 : 0));
  EnvPlan E;
  STCHK(plan_envs(h, eb, reinterpret_cast<double2*>(sc + o_t), tel, E));
  if (o_list + E.pk.total > cap)
    return fail(MPS_E_ARG, "mps_norm_noalloc: bond dimension %d needs %zu bytes of scratch, the limit is %zu",
                maxdim, o_list + E.pk.total, cap);
  // pageable staging on the host: the copy completes before the call returns
  std::vector<char> stage(E.pk.total);
  E.pk.write(stage.data());
  HIPCHK(hipMemcpyAsync(sc + o_list, stage.data(), E.pk.total, hipMemcpyHostToDevice, h->st));
  STCHK(launch_envs(h, eb, E, sc + o_list));
  double2 res = make_double2(0.0, 0.0);
  HIPCHK(hipMemcpyAsync(&res, eb[L], sizeof(double2), hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  *norm2 = res.x;
  return MPS_OK;
}

}  // extern "C"

namespace {

// Samples per round of the sampler (bounds its buffers: about 10 vectors of
// the largest charge block per sample).
constexpr int kSampleChunk = 8192;

// `cnt` samples with the environments eb already built: one round per mode,
// from the last to the first (see sample.hip).  Each round is planned on the
// device from the samples' charge positions, so all rounds are enqueued
// without waiting and the host synchronises once at the end.
mps_status sample_chunk(mps_state* h, const std::vector<double2*>& eb, int cnt, const double* uniforms,
                        int* occ, double* prob) {
  const int L = h->L, d = h->d, zn = h->mod;
  // fixed candidate tables of every round and upper bounds of its grids
  int maxblk = 1, maxq = 1;
  for (int b = 0; b <= L; ++b) {
    for (int c : h->bonds[b].count) maxblk = std::max(maxblk, c);
    maxq = std::max(maxq, (int)h->bonds[b].charge.size());
  }
  if (maxq > kMaxSampleCharges) return fail(MPS_E_ARG, "more than %d charges on a bond", kMaxSampleCharges);
  std::vector<SampleCand> cand;
  std::vector<size_t> cand_off(L);
  std::vector<int> ub_gemm(L), ub_pick(L);
  std::vector<long long> ub_elems(L);
  const long long ctiles = (cnt + kGemmTile - 1) / kGemmTile;
  for (int s = 0; s < L; ++s) {
    const Bond& B0 = h->bonds[s];
    const Bond& B1 = h->bonds[s + 1];
    cand_off[s] = cand.size();
    long long maxrt = 0, sumrt = 0;
    int maxnc = 1;
    for (size_t q = 0; q < B1.charge.size(); ++q) {
      const int c = B1.charge[q];
      SampleCand sc{};
      sc.nc = B1.count[q];
      sc.off1 = B1.off[q];
      long long rt = 0;
      for (int i = 0; i < d; ++i) {
        const int c2 = zn ? (c + i) % zn : c + h->rule.step[i];
        const int ri = B0.find(c2);
        if (ri < 0) continue;
        sc.loc[sc.nout] = i;
        sc.pos[sc.nout] = ri;
        sc.nr[sc.nout] = B0.count[ri];
        sc.off0[sc.nout] = B0.off[ri];
        rt += (B0.count[ri] + kGemmTile - 1) / kGemmTile;
        ++sc.nout;
      }
      maxrt = std::max(maxrt, rt);
      sumrt += rt;
      maxnc = std::max(maxnc, sc.nc);
      cand.push_back(sc);
    }
    // sum_q rt_q ceil(ng_q / T) <= max_q rt_q ceil(cnt / T) + sum_q rt_q
    const long long ub = maxrt * ctiles + sumrt;
    if (ub > INT_MAX) return fail(MPS_E_ARG, "sampling round %d too large", s);
    ub_gemm[s] = (int)ub;
    ub_pick[s] = (cnt + 15) / 16 + (int)B1.charge.size();
    ub_elems[s] = (long long)maxnc * cnt;
  }
  const size_t vec = (size_t)maxblk * cnt;        // one vector of the largest block per sample
  Packer pk;
  const size_t o_u = pk.add(nullptr, (size_t)cnt * L * sizeof(double));
  const size_t o_occ = pk.add(nullptr, (size_t)cnt * L * sizeof(int));
  const size_t o_pr = pk.add(nullptr, (size_t)cnt * sizeof(double));
  const size_t o_pos = pk.add(nullptr, (size_t)cnt * sizeof(int));
  const size_t o_cnt = pk.add(nullptr, sizeof(SampleCounts));
  const size_t o_cand = pk.add(nullptr, cand.size() * sizeof(SampleCand));
  const size_t o_slot = pk.add(nullptr, vec * sizeof(double2));
  const size_t o_v = pk.add(nullptr, vec * sizeof(double2));
  const size_t o_w = pk.add(nullptr, (size_t)d * vec * sizeof(double2));
  const size_t o_x = pk.add(nullptr, (size_t)d * vec * sizeof(double2));
  const size_t o_ids = pk.add(nullptr, (size_t)cnt * sizeof(int));
  const size_t o_grp = pk.add(nullptr, (size_t)maxq * sizeof(SampleGroup));
  const size_t o_g1 = pk.add(nullptr, (size_t)maxq * kMaxD * sizeof(GemmWork));
  const size_t o_g2 = pk.add(nullptr, (size_t)maxq * kMaxD * sizeof(GemmWork));
  STCHK(ensure(h, h->samp, pk.total));
  // inputs, laid out as on the device from o_u to o_slot (the initial vector 1
  // of every sample, on the single charge of bond L, goes to row 0 of the
  // slots), through the sampler's own pinned buffer (whose last use, the
  // previous chunk's results, has been waited for)
  const size_t head = o_slot + (size_t)cnt * sizeof(double2);
  const size_t tail_out =
      align256((size_t)cnt * L * sizeof(int)) + align256((size_t)cnt * sizeof(double)) + sizeof(SampleCounts);
  STCHK(ensure_pin(h->stage_samp, std::max(head, tail_out)));
  char* stg = static_cast<char*>(h->stage_samp.p);
  std::memset(stg, 0, head);
  std::memcpy(stg + o_u, uniforms, (size_t)cnt * L * sizeof(double));
  double* pones = reinterpret_cast<double*>(stg + o_pr);
  double2* vones = reinterpret_cast<double2*>(stg + o_slot);
  for (int j = 0; j < cnt; ++j) {
    pones[j] = 1.0;
    vones[j] = make_double2(1.0, 0.0);
  }
  std::memcpy(stg + o_cand, cand.data(), cand.size() * sizeof(SampleCand));
  char* dev = static_cast<char*>(h->samp.p);
  HIPCHK(hipMemcpyAsync(dev, stg, head, hipMemcpyHostToDevice, h->st));
  int* d_pos = reinterpret_cast<int*>(dev + o_pos);
  SampleCounts* d_cnt = reinterpret_cast<SampleCounts*>(dev + o_cnt);
  double2* slots = reinterpret_cast<double2*>(dev + o_slot);
  double2* vbuf = reinterpret_cast<double2*>(dev + o_v);
  double2* wbuf = reinterpret_cast<double2*>(dev + o_w);
  double2* xbuf = reinterpret_cast<double2*>(dev + o_x);
  int* d_ids = reinterpret_cast<int*>(dev + o_ids);
  SampleGroup* d_grp = reinterpret_cast<SampleGroup*>(dev + o_grp);
  GemmWork* d_g1 = reinterpret_cast<GemmWork*>(dev + o_g1);
  GemmWork* d_g2 = reinterpret_cast<GemmWork*>(dev + o_g2);
  const SampleCand* d_cand = reinterpret_cast<const SampleCand*>(dev + o_cand);
  for (int s = L - 1; s >= 0; --s) {
    const Bond& B0 = h->bonds[s];
    const Bond& B1 = h->bonds[s + 1];
    const int nq = (int)B1.charge.size();
    HIPCHK(launch_sample_plan(d_cand + cand_off[s], nq, d_pos, cnt, h->site[s], B1.dim(), eb[s], B0.dim(), vbuf,
                              wbuf, xbuf, d_ids, d_grp, d_g1, d_g2, d_cnt, h->st));
    HIPCHK(launch_sample_gather(d_grp, nq, ub_elems[s], d_ids, slots, cnt, vbuf, h->st));
    HIPCHK(launch_zgemm(d_g1, nq * kMaxD, ub_gemm[s], h->st, &d_cnt->nt1));
    HIPCHK(launch_zgemm(d_g2, nq * kMaxD, ub_gemm[s], h->st, &d_cnt->nt2));
    HIPCHK(launch_sample_pick(d_grp, nq, ub_pick[s], d_ids, wbuf, xbuf, reinterpret_cast<const double*>(dev + o_u), L,
                              s, slots, cnt, reinterpret_cast<int*>(dev + o_occ), reinterpret_cast<double*>(dev + o_pr),
                              d_pos, d_cnt, h->st));
  }
  // results back through pinned memory (the staging buffer, sized for them
  // above; the copies are ordered after the upload on the stream):
  // occupations, probabilities, the flag
  int* h_occ = reinterpret_cast<int*>(stg);
  double* h_pr = reinterpret_cast<double*>(stg + align256((size_t)cnt * L * sizeof(int)));
  SampleCounts* h_cnt = reinterpret_cast<SampleCounts*>(stg + align256((size_t)cnt * L * sizeof(int)) +
                                                         align256((size_t)cnt * sizeof(double)));
  HIPCHK(hipMemcpyAsync(h_occ, dev + o_occ, (size_t)cnt * L * sizeof(int), hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipMemcpyAsync(h_pr, dev + o_pr, (size_t)cnt * sizeof(double), hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipMemcpyAsync(h_cnt, d_cnt, sizeof(SampleCounts), hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  if (h_cnt->failed) return fail(MPS_E_NUMERIC, "a sample met a vanished or non-finite marginal");
  std::memcpy(occ, h_occ, (size_t)cnt * L * sizeof(int));
  std::memcpy(prob, h_pr, (size_t)cnt * sizeof(double));
  return MPS_OK;
}

}  // namespace

extern "C" {

mps_status mps_sample(mps_t h, int count, const double* uniforms, int* occ, double* prob) {
  if (!valid_handle(h)) return fail(MPS_E_ARG, "invalid handle");
  if (count < 0) return fail(MPS_E_ARG, "negative count");
  if (count == 0) return MPS_OK;
  if (!uniforms || !occ) return fail(MPS_E_ARG, "uniforms and occ are required");
  const int L = h->L;
  for (size_t k = 0; k < (size_t)count * L; ++k)
    if (!(uniforms[k] >= 0.0 && uniforms[k] < 1.0)) return fail(MPS_E_ARG, "uniform %zu outside [0, 1)", k);
  size_t etot = 0;
  std::vector<size_t> eoff(L + 1);
  for (int b = 0; b <= L; ++b) {
    eoff[b] = etot;
    etot += (size_t)h->bonds[b].dim() * h->bonds[b].dim();
  }
  STCHK(ensure(h, h->envs, etot * sizeof(double2)));
  std::vector<double2*> eb(L + 1);
  for (int b = 0; b <= L; ++b) eb[b] = static_cast<double2*>(h->envs.p) + eoff[b];
  // the environments run while the host prepares the first chunk (the
  // sampler stages through its own pinned buffer, so nothing waits for them)
  size_t tail = 0;
  STCHK(left_envs(h, eb, 0, &tail));
  std::vector<double> pr(count);
  mps_status st = MPS_OK;
  for (int c0 = 0; c0 < count && st == MPS_OK; c0 += kSampleChunk) {
    const int cnt = std::min(kSampleChunk, count - c0);
    st = sample_chunk(h, eb, cnt, uniforms + (size_t)c0 * L, occ + (size_t)c0 * L, pr.data() + c0);
  }
  // the environments and the round buffers are as large as the state: give them back
  (void)hipStreamSynchronize(h->st);
  dfree(h, h->envs.p);
  h->envs.p = nullptr;
  h->envs.cap = 0;
  dfree(h, h->samp.p);
  h->samp.p = nullptr;
  h->samp.cap = 0;
  if (st != MPS_OK) return st;
  if (prob) std::memcpy(prob, pr.data(), (size_t)count * sizeof(double));
  return MPS_OK;
}

mps_status mps_bond_sectors(mps_t h, int bond, int cap, int* nsec, int* charge, int* count) {
  if (!valid_handle(h)) return fail(MPS_E_ARG, "invalid handle");
  if (bond < 0 || bond > h->L) return fail(MPS_E_ARG, "bond %d outside 0..L", bond);
  const Bond& B = h->bonds[bond];
  if (nsec) *nsec = (int)B.charge.size();
  if ((int)B.charge.size() > cap) return fail(MPS_E_ARG, "capacity %d < %zu sectors", cap, B.charge.size());
  for (size_t i = 0; i < B.charge.size(); ++i) {
    if (charge) charge[i] = B.charge[i];
    if (count) count[i] = B.count[i];
  }
  return MPS_OK;
}

mps_status mps_bond_lambda(mps_t h, int bond, int cap, int* n, double* lambda) {
  if (!valid_handle(h)) return fail(MPS_E_ARG, "invalid handle");
  if (bond < 0 || bond > h->L) return fail(MPS_E_ARG, "bond %d outside 0..L", bond);
  const int dim = h->bonds[bond].dim();
  if (n) *n = dim;
  if (dim > cap) return fail(MPS_E_ARG, "capacity %d < dimension %d", cap, dim);
  if (!lambda) return fail(MPS_E_ARG, "lambda is NULL");
  HIPCHK(hipMemcpyAsync(lambda, h->lam[bond], (size_t)dim * sizeof(double), hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  return MPS_OK;
}

mps_status mps_site_tensor(mps_t h, int site, size_t cap, int* rows, int* cols, mps_z* out) {
  if (!valid_handle(h)) return fail(MPS_E_ARG, "invalid handle");
  if (site < 0 || site >= h->L) return fail(MPS_E_ARG, "site %d outside 0..L-1", site);
  const int r = h->bonds[site].dim(), c = h->bonds[site + 1].dim();
  if (rows) *rows = r;
  if (cols) *cols = c;
  if ((size_t)r * c > cap) return fail(MPS_E_ARG, "capacity too small");
  if (!out) return fail(MPS_E_ARG, "out is NULL");
  HIPCHK(hipMemcpyAsync(out, h->site[site], (size_t)r * c * sizeof(double2), hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  return MPS_OK;
}

mps_status mps_last_leaks(mps_t h, int cap, int* n, double* leak) {
  if (!valid_handle(h)) return fail(MPS_E_ARG, "invalid handle");
  const int cnt = (int)h->last_leak.size();
  if (n) *n = cnt;
  if (cnt > cap) return fail(MPS_E_ARG, "capacity %d < %d gates", cap, cnt);
  if (cnt && !leak) return fail(MPS_E_ARG, "leak is NULL");
  for (int i = 0; i < cnt; ++i) leak[i] = h->last_leak[i];
  return MPS_OK;
}

mps_status mps_set_timing(mps_t h, int on) {
  if (!valid_handle(h)) return fail(MPS_E_ARG, "invalid handle");
  HIPCHK(hipStreamSynchronize(h->st));
  STCHK(drain_events(h));
  h->timing = on != 0;
  return MPS_OK;
}

mps_status mps_get_stats(mps_t h, mps_stats* s) {
  if (!valid_handle(h) || !s) return fail(MPS_E_ARG, "invalid handle or NULL stats");
  HIPCHK(hipStreamSynchronize(h->st));
  STCHK(drain_events(h));
  *s = h->stats;
  return MPS_OK;
}

mps_status mps_reset_stats(mps_t h) {
  if (!valid_handle(h)) return fail(MPS_E_ARG, "invalid handle");
  HIPCHK(hipStreamSynchronize(h->st));
  STCHK(drain_events(h));
  h->stats = mps_stats{};
  h->stats.min_margin = INFINITY;
  return MPS_OK;
}

mps_status mps_sync(mps_t h) {
  if (!valid_handle(h)) return fail(MPS_E_ARG, "invalid handle");
  HIPCHK(hipStreamSynchronize(h->st));
  return drain_events(h);
}

}  // extern "C"
