// Per-sector SVD of the two-site update (Sec. II: the SVD of Theta split into
// its middle-charge blocks): blocked one-sided (Hestenes) Jacobi in FP64 on
// every Theta(m) of a batch, one launch per round-robin step.
#include "device_util.h"
#include "kernels.h"

namespace u1mps {

// ---------------------------------------------------------------------------
// One-sided (Hestenes) Jacobi SVD of Theta(m), blocked.
//
// The SVD runs on the min(r, c) vectors of length max(r, c): the rows of
// Theta when r <= c, else its columns (the theta kernel stores a tall sector
// transposed).  A vector pair (x, y) with alpha = |x|^2, beta = |y|^2,
// gamma = <x, y> is made orthogonal by the rotation
//   zeta = (beta - alpha) / (2|gamma|), t = sgn(zeta) / (|zeta| + sqrt(1 + zeta^2)),
//   c = 1/sqrt(1 + t^2), s = c t, w = s gamma/|gamma|,
//   x' = c x - w y,  y' = conj(w) x + c y,
// applied while |gamma| > tol sqrt(alpha beta) and |gamma| is above the
// rounding floor of the sector.  Vectors are grouped in blocks of kJB; a
// round-robin (circle method) schedule over the blocks pairs every two
// blocks once per sweep.  For a block pair the workgroup forms the Gram
// matrix G = X X^H of its 2 kJB vectors, applies rotations to G
// (G <- U G U^H; a bounded number of sweeps over its pairs, not necessarily
// to tolerance), accumulating W = prod U, and rotates the vectors, X <- W X.
// Convergence is always judged on a Gram matrix freshly formed from the
// vectors, so the stopping rule is the same pairwise-cosine test as for the
// unblocked method; the outer sweeps carry the iteration to it.
// With J the product of all rotations, J X = S Y with orthonormal rows Y:
//   wide (X = Theta):    V^dagger = Y, the normalised vectors;
//   tall (X = Theta^T):  V^dagger = conj(J), accumulated in A (c x c) from I.
__device__ __forceinline__ void rr_pair(int step, int k, int np, int& i, int& j) {
  const int q = np - 1;
  if (k == 0) {
    i = step % q;
    j = q;
  } else {
    i = (step + k) % q;
    j = (step - k + q) % q;
  }
}

// a' = c a - w b ; b' = conj(w) a + c b, with w = wr + i wi
__device__ __forceinline__ void rot_pair(double2& a, double2& b, double c, double wr, double wi) {
  const double2 x = a, y = b;
  a.x = c * x.x - (wr * y.x - wi * y.y);
  a.y = c * x.y - (wr * y.y + wi * y.x);
  b.x = (wr * x.x + wi * x.y) + c * y.x;
  b.y = (wr * x.y - wi * x.x) + c * y.y;
}

__device__ __forceinline__ bool jac_rotation(double al, double be, double gr, double gi, double tol,
                                             double floor_g, double& c, double& wr, double& wi) {
  // test on squares: |gamma|^2 > tol^2 alpha beta and |gamma| > floor
  const double g2 = gr * gr + gi * gi;
  const bool rot = (g2 > tol * tol * al * be) && (g2 > floor_g * floor_g);
  // with delta = beta - alpha, r = sqrt(delta^2 + 4|gamma|^2), D = |delta| + r:
  // c = D / E, w = 2 sgn(delta) gamma / E with E^2 = D^2 + 4|gamma|^2 (= 2 r D)
  // -- the rotation t = sgn(zeta) / (|zeta| + sqrt(1 + zeta^2)),
  // zeta = delta / (2|gamma|), c = 1/sqrt(1 + t^2), w = c t gamma/|gamma|.
  // Only the angle depends on r, so r is taken from the hardware reciprocal
  // square root without refinement (relative error far below what a sweep
  // needs: the pair is left with a cosine of that order instead of 0); E is
  // formed from the D actually used and inverted to full precision, so
  // c^2 + |w|^2 = 1 to rounding.  Computed without branches (the identity is
  // selected when the pair is below the thresholds), so that the rotations of
  // several pairs interleave.
  const double delta = be - al;
  const double x = fma(delta, delta, 4.0 * g2);
  const double r = x * __builtin_amdgcn_rsq(x);
  const double D = fabs(delta) + r;
  const double inv = rsqrt(fma(D, D, 4.0 * g2));
  const double sg = delta >= 0.0 ? 2.0 * inv : -2.0 * inv;
  c = rot ? D * inv : 1.0;
  wr = rot ? sg * gr : 0.0;
  wi = rot ? sg * gi : 0.0;
  return rot;
}

// Default threshold: (vector length) * eps, but never below 2 * kJP * eps,
// the rounding level of the kJP-term combinations X <- W X that rotate a
// block pair (short vectors would otherwise be held to a test they cannot
// pass).
__device__ __forceinline__ double jac_tol(double tol_opt, int len) {
  return tol_opt > 0.0 ? tol_opt : (double)max(len, 2 * kJP) * DBL_EPSILON;
}

// One workgroup of kJacRowThreads per sector: reset state, vector norms (a
// wavefront per vector), identity order, squared Frobenius norm (the
// wavefronts' partial sums added in wavefront order), A = I.
constexpr int kJacRowThreads = 1024;

__global__ void __launch_bounds__(kJacRowThreads)
jacobi_init(const SectorWork* __restrict__ secs, const int* __restrict__ list,
            const double2* __restrict__ theta, double2* __restrict__ accbuf,
            JacobiOut* __restrict__ st, int* __restrict__ perm, double* __restrict__ norm2) {
  constexpr int kWaves = kJacRowThreads / 64;
  __shared__ double wsum[kWaves];
  const int sid = list[blockIdx.x];
  const SectorWork sw = secs[sid];
  const bool tall = sw.tall != 0;
  const int n = tall ? sw.c : sw.r;
  const int len = tall ? sw.r : sw.c;
  const double2* x = theta + sw.off;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (tall) {
    double2* a = accbuf + sw.acc;
    for (int e = threadIdx.x; e < n * n; e += blockDim.x)
      a[e] = make_double2((e / n) == (e % n) ? 1.0 : 0.0, 0.0);
  }
  double f = 0.0;
  for (int i = wave; i < n; i += kWaves) {
    const double2* xi = x + (size_t)i * len;
    double ss = 0.0;
    for (int col = lane; col < len; col += 64) {
      const double2 v = xi[col];
      ss = fma(v.x, v.x, fma(v.y, v.y, ss));
    }
    ss = wave_sum(ss);
    if (lane == 0) {
      norm2[sw.sig + i] = ss;
      perm[sw.sig + i] = i;
    }
    f += ss;
  }
  if (lane == 0) wsum[wave] = f;
  __syncthreads();
  if (threadIdx.x == 0) {
    JacobiOut o;
    o.sweeps = 0;
    o.rotations = 0;
    o.converged = n < 2 ? 1 : 0;
    o.rot3[0] = o.rot3[1] = o.rot3[2] = 0;
    o.gram_units = 0;
    o.apply_units = 0;
    double fro2 = 0.0;
    for (int w = 0; w < kWaves; ++w) fro2 += wsum[w];
    o.fro2 = fro2;
    st[sid] = o;
  }
}

// Column chunks of the kJP rows vrow[r] (-1 = absent) of a row-major matrix
// with row length len.  A chunk is 32 columns; each of the 256 threads moves
// kJChunkRegs of its elements (rows 8 k + tid / 32, column tid % 32), so a
// wavefront reads two contiguous 512-byte row segments per load.  Absent
// rows and columns past len read as 0 and issue no load.
constexpr int kJChunkRegs = kJP * 32 / 256;

__device__ __forceinline__ void jac_fetch(double2 (&v)[kJChunkRegs], const double2* __restrict__ x,
                                          int len, int c0, const int* vrow) {
  const int cc = threadIdx.x & 31, col = c0 + cc;
#pragma unroll
  for (int k = 0; k < kJChunkRegs; ++k) {
    const int row = vrow[8 * k + (threadIdx.x >> 5)];
    v[k] = make_double2(0.0, 0.0);
    if (row >= 0 && col < len) v[k] = x[(size_t)row * len + col];
  }
}

__device__ __forceinline__ void jac_stage(double2 (*xs)[kJP + 2], const double2 (&v)[kJChunkRegs]) {
  const int cc = threadIdx.x & 31;
#pragma unroll
  for (int k = 0; k < kJChunkRegs; ++k) xs[8 * k + (threadIdx.x >> 5)][cc] = v[k];
}

// Runs body(c0) for every chunk [c0, c0 + 32) of the rows, with the chunk
// staged in xs.  Two chunks are in flight in registers while the body works
// on the staged one, so the loads of chunk c0 + 64 overlap the body of c0.
// The body may overwrite columns [c0, c0 + 32) of x (the loads in flight
// are of later columns).
template <class Body>
__device__ __forceinline__ void jac_chunk_loop(double2 (*xs)[kJP + 2], const double2* x, int len,
                                               const int* vrow, Body&& body) {
  double2 ra[kJChunkRegs], rb[kJChunkRegs];
  jac_fetch(ra, x, len, 0, vrow);
  jac_fetch(rb, x, len, 32, vrow);
  for (int c0 = 0; c0 < len; c0 += 64) {
    jac_stage(xs, ra);
    __syncthreads();
    jac_fetch(ra, x, len, c0 + 64, vrow);
    body(c0);
    __syncthreads();
    if (c0 + 32 >= len) break;
    jac_stage(xs, rb);
    __syncthreads();
    jac_fetch(rb, x, len, c0 + 96, vrow);
    body(c0 + 32);
    __syncthreads();
  }
}

// X_IJ <- W X_IJ for one row-major matrix (rows of length len), in column
// chunks of 32, on the matrix cores: wave w computes the 16 x 16 output
// quadrant (rows 16 (w / 2), columns 16 (w % 2)) of each chunk as three real
// products per k-step (below).
__device__ void jac_apply(double2 (*xs)[kJP + 2], double2 (*ws)[kJP + 2], double2* __restrict__ x,
                          int len, const int* vrow) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int R = (wave >> 1) * 16, Cq = (wave & 1) * 16;
  const int li = lane & 15, lk = lane >> 4;
  jac_chunk_loop(xs, x, len, vrow, [&](int c0) {
    // three real products (Gauss): P1 = Wr Xr, P2 = Wi Xi, P3 = (Wr + Wi)(Xr + Xi);
    // Re = P1 - P2, Im = P3 - P1 - P2 -- three independent accumulator chains
    v4d p1 = {0.0, 0.0, 0.0, 0.0}, p2 = {0.0, 0.0, 0.0, 0.0}, p3 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k0 = 0; k0 < kJP; k0 += 4) {
      const double2 wv = ws[R + li][k0 + lk];      // A = W[R + i][k]
      const double2 xv = xs[k0 + lk][Cq + li];     // B = X[k][C + j]
      p1 = mfma16x16x4(wv.x, xv.x, p1);
      p2 = mfma16x16x4(wv.y, xv.y, p2);
      p3 = mfma16x16x4(wv.x + wv.y, xv.x + xv.y, p3);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int v = vrow[R + 4 * r + lk];
      const int col = c0 + Cq + li;
      if (v >= 0 && col < len) x[(size_t)v * len + col] = make_double2(p1[r] - p2[r], p3[r] - p1[r] - p2[r]);
    }
  });
}

// Gram matrix G = X X^H of the kJP rows into gs, on the matrix cores, with
// three real products: Gr = Xr Xr^T + Xi Xi^T (symmetric) and Gi = M - M^T
// with M = Xi Xr^T.  Waves 0, 1, 2 form the Gr quadrants (0,0), (0,16),
// (16,16) and the same quadrants of M; wave 3 forms M's quadrant (16,0).
// Gr's diagonal quadrants give both triangles with different rounding;
// every decision must see one value per pair, so gs is made exactly
// Hermitian from its upper triangle.  M passes through xs.
__device__ void jac_gram(double2 (*xs)[kJP + 2], double2 (*gs)[kJP + 2], const double2* x, int len,
                         const int* vrow) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int P = wave >= 2 ? 16 : 0, Q = (wave == 1 || wave == 2) ? 16 : 0;
  const int li = lane & 15, lk = lane >> 4;
  const bool has_gr = wave < 3;
  v4d gra = {0.0, 0.0, 0.0, 0.0}, grb = {0.0, 0.0, 0.0, 0.0}, mm = {0.0, 0.0, 0.0, 0.0};
  jac_chunk_loop(xs, x, len, vrow, [&](int) {
#pragma unroll
    for (int k0 = 0; k0 < 32; k0 += 4) {
      const double2 av = xs[P + li][k0 + lk];     // A = X[P + i][k]
      const double2 bv = xs[Q + li][k0 + lk];     // B = X[Q + j][k] (transposed)
      if (has_gr) {
        gra = mfma16x16x4(av.x, bv.x, gra);
        grb = mfma16x16x4(av.y, bv.y, grb);
      }
      mm = mfma16x16x4(av.y, bv.x, mm);
    }
  });
  // the loop ended on a barrier: xs is free
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    if (has_gr) gs[P + 4 * r + lk][Q + li] = make_double2(gra[r] + grb[r], 0.0);
    xs[P + 4 * r + lk][Q + li] = make_double2(mm[r], 0.0);
  }
  __syncthreads();
  for (int e = tid; e < kJP * kJP; e += blockDim.x) {
    const int r = e / kJP, c = e % kJP;
    if (r < c) {
      const double2 g = make_double2(gs[r][c].x, xs[r][c].x - xs[c][r].x);
      gs[r][c] = g;
      gs[c][r] = cconj(g);
    }
  }
}

// Pair k of round-robin step s over the kJP rows of a block pair, as (p, q)
// with p < q: the rotation always reads the upper-triangle entry.
__device__ __forceinline__ void jac_pair_ordered(int s, int k, int& p, int& q) {
  int i, j;
  rr_pair(s, k, kJP, i, j);
  p = min(i, j);
  q = max(i, j);
}

// Pair k of round-robin step s over the kJP rows as (p, q), p < q: the pairs
// of rr_pair(s, k, kJP), (s + k, s - k) mod (kJP - 1) and (s, kJP - 1) for
// k = 0, computed with selects instead of divisions (s < kJP - 1, k < kJP / 2).
__device__ __forceinline__ void jac_pair_fast(int s, int k, int& p, int& q) {
  int i = s + k;
  i = i >= kJP - 1 ? i - (kJP - 1) : i;
  int j = s - k;
  j = j < 0 ? j + (kJP - 1) : j;
  j = k == 0 ? kJP - 1 : j;
  p = min(i, j);
  q = max(i, j);
}

// Workgroup-wide OR of a predicate with one barrier: lane 0 of each
// wavefront publishes its wavefront's ballot in slot `parity` of flags, which
// alternates between calls, so a slot is rewritten only after every thread
// has passed the barrier of the call in between.  Every thread of the
// workgroup must make the same sequence of calls.
__device__ __forceinline__ bool block_any(int pred, int4* flags, int& parity) {
  const bool w = __ballot(pred) != 0ull;
  int* f = reinterpret_cast<int*>(flags + parity);
  if ((threadIdx.x & 63) == 0) f[threadIdx.x >> 6] = w ? 1 : 0;
  __syncthreads();
  const int4 v = flags[parity];
  parity ^= 1;
  return (v.x | v.y | v.z | v.w) != 0;
}

// True if the pair (p, q) of a Gram matrix with diagonal alpha, beta and
// off-diagonal gamma is above the rotation threshold (the test of
// jac_rotation without computing the rotation).
__device__ __forceinline__ bool jac_needs(double al, double be, double2 g, double tol, double floor_g) {
  const double g2 = g.x * g.x + g.y * g.y;
  return g2 > tol * tol * al * be && g2 > floor_g * floor_g;
}

// True if any off-diagonal pair of the Hermitian gs is above the threshold:
// thread t checks the upper-triangle entries of its 2 x 2 block (rows
// 2 (t / 16), columns 2 (t % 16)).  Uniform across the workgroup.
__device__ __forceinline__ bool jac_any_above(double2 (*gs)[kJP + 2], double tol, double floor_g,
                                              int4* anyf, int& parity) {
  const int p0 = 2 * (threadIdx.x >> 4), q0 = 2 * (threadIdx.x & 15);
  int f = 0;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int p = p0 + i, q = q0 + j;
      if (p < q && jac_needs(gs[p][p].x, gs[q][q].x, gs[p][q], tol, floor_g)) f = 1;
    }
  return block_any(f, anyf, parity);
}

// Rotations of the Gram matrix gs (in LDS): up to max_inner sweeps, fewer if
// no pair exceeds the threshold any more; W accumulates the product.  The
// caller has established that some pair is above it.  A round-robin step rotates 16 disjoint pairs at
// once, G <- U G U^H and W <- U W with U block diagonal over the pairs.
// Thread t = 16 A + B owns the 2 x 2 blocks (rows of pair A) x (columns of
// pair B): it computes the rotations of pairs A and B itself from the
// current G, writes its rotated G block into the other buffer (g1, the
// staging tile, idle during the eig) and updates its W block in place, so a
// step needs one barrier and no exchange of rotations.  After each sweep one
// parallel test over all pairs replaces the sweep that would find nothing to
// rotate (it would leave G and W unchanged); after the last allowed sweep the
// test is skipped.  The final G is left in gs.
__device__ void jac_gram_eig(double2 (*gs)[kJP + 2], double2 (*g1)[kJP + 2], double2 (*ws)[kJP + 2],
                             double tol, double floor_g, int max_inner, int4* anyf, int& parity) {
  const int tid = threadIdx.x;
  const int A = tid >> 4, B = tid & 15;
  double2 (*cur)[kJP + 2] = gs;
  double2 (*nxt)[kJP + 2] = g1;
  for (int inner = 0; inner < max_inner; ++inner) {
    for (int s2 = 0; s2 < kJP - 1; ++s2) {
      int pa, qa, pb, qb;
      jac_pair_fast(s2, A, pa, qa);
      jac_pair_fast(s2, B, pb, qb);
      // every LDS read of the step first, so that their latencies overlap
      const double2 ga = cur[pa][qa], gb = cur[pb][qb];
      const double apa = cur[pa][pa].x, aqa = cur[qa][qa].x, apb = cur[pb][pb].x, aqb = cur[qb][qb].x;
      double2 g00 = cur[pa][pb], g01 = cur[pa][qb], g10 = cur[qa][pb], g11 = cur[qa][qb];
      double2 w00 = ws[pa][pb], w01 = ws[pa][qb], w10 = ws[qa][pb], w11 = ws[qa][qb];
      double ca, wra, wia, cb, wrb, wib;
      jac_rotation(apa, aqa, ga.x, ga.y, tol, floor_g, ca, wra, wia);
      jac_rotation(apb, aqb, gb.x, gb.y, tol, floor_g, cb, wrb, wib);
      // rows pa, qa: U from the left, also on W; columns pb, qb: U^H from the
      // right (an identity rotation leaves a block exactly as it was)
      rot_pair(g00, g10, ca, wra, wia);
      rot_pair(g01, g11, ca, wra, wia);
      rot_pair(w00, w10, ca, wra, wia);
      rot_pair(w01, w11, ca, wra, wia);
      rot_pair(g00, g01, cb, wrb, -wib);
      rot_pair(g10, g11, cb, wrb, -wib);
      ws[pa][pb] = w00; ws[pa][qb] = w01; ws[qa][pb] = w10; ws[qa][qb] = w11;
      nxt[pa][pb] = g00; nxt[pa][qb] = g01; nxt[qa][pb] = g10; nxt[qa][qb] = g11;
      // every read of cur in this step precedes the barrier, so the next step may overwrite it
      __syncthreads();
      double2 (*t)[kJP + 2] = cur;
      cur = nxt;
      nxt = t;
    }
    if (inner + 1 < max_inner && !jac_any_above(cur, tol, floor_g, anyf, parity)) break;
  }
  // a sweep has an odd number of steps: an odd sweep count leaves G in g1
  if (cur != gs)
    for (int e = tid; e < kJP * kJP; e += blockDim.x) gs[e / kJP][e % kJP] = cur[e / kJP][e % kJP];
  __syncthreads();
}

// One round-robin step for every active sector: one workgroup per block pair.
//
// A block pair that fails the convergence test is rotated once per visit,
// with one of two thresholds.  While some pair of its Gram matrix is above
// kJacLoose relative off-diagonal (and above the Gram's own rounding level,
// kJacNoise * eps * max diagonal), the rotations of G use those coarse
// thresholds: rotations of G itself carry errors of order eps * max|G|, which
// would leave the smallest vectors of the pair with cosines of
// eps * s_max^2 / (s_p s_q) if pursued further.  Only a Gram matrix with
// nothing above the coarse thresholds is rotated to the full tolerance; it is
// then nearly diagonal, its rotations are small and their errors are relative
// to each vector's own norm.  A visit that rotated at the coarse thresholds
// ends there: the next sweep forms the Gram matrix afresh.
constexpr double kJacLoose = 1e-8;
constexpr double kJacNoise = 64.0;

// Where the workgroup of block pair w (blocks of JB vectors) stands in step
// launch t, and its rows.  Lockstep launches (desync 0) run step t of every
// sector's current sweep; the sweep ends in kernels of their own
// (jacobi_sweep_end, jacobi_sort).  Desynchronised launches run, for every
// sector, its own step s = t mod (nb - 1) of its sweep t div (nb - 1), so a
// sector with few blocks starts its next sweep without waiting for the
// largest one.  There, at s = 0 of every sweep after the first, the sector's
// workgroups first close the previous sweep as jacobi_sweep_end would (pair
// 0 keeps the books and counts the sector out of ctr[0], into ctr[1] when it
// stops unconverged at the sweep limit) and take their rows in the order
// jacobi_sort would write (descending norm, index order among equals;
// scratch holds the n norms), writing that order for the sweep's later steps;
// the sweep's rotation count is rot3[sweep % 3], and its visits leave the
// vector norms in buffer sweep % 2 of norm2 (nstride doubles apart), so that
// the first step of the next sweep sorts on the other buffer while visits of
// that step write theirs.  Sets the slot, the norm buffer nbuf, the rows
// vrow[0 .. 2 JB) (-1: absent) and returns the number present, or -1
// (uniform) when the pair has nothing to do.
template <int JB>
__device__ int jac_setup(const JacobiPairWork& w, const SectorWork& sw, int sid, int t, int desync, int blocked,
                         int* __restrict__ ctr, JacobiOut* __restrict__ st, int* __restrict__ perm,
                         const double* __restrict__ norm2, long long nstride, double* scratch, int* vrow, int& slot,
                         int& nbuf) {
  const int tid = threadIdx.x;
  const int n = sw.tall ? sw.c : sw.r;
  int s = t, sweep = 0;
  if (desync) {
    s = t % (w.nb - 1);
    sweep = t / (w.nb - 1);
    if (sweep > blocked || (sweep == blocked && s > 0)) return -1;
  } else if (s >= w.nb - 1) {
    return -1;
  }
  slot = desync ? sweep % 3 : 0;
  nbuf = desync ? sweep & 1 : 0;
  int bi, bj;
  rr_pair(s, w.k, w.nb, bi, bj);
  const int vI = bi * JB, vJ = bj * JB;
  const int nI = max(0, min(JB, n - vI)), nJ = max(0, min(JB, n - vJ));
  if (desync && s == 0 && sweep > 0) {
    const int rot = st[sid].rot3[(sweep - 1) % 3];
    const bool done = rot == 0 || sweep >= blocked;
    if (w.k == 0 && tid == 0) {
      JacobiOut* o = st + sid;
      o->sweeps += 1;
      o->rotations += rot;
      if (rot == 0) o->converged = 1;
      if (done) {
        atomicSub(&ctr[0], 1);
        if (rot != 0) atomicAdd(&ctr[1], 1);
      } else {
        o->rot3[(sweep + 1) % 3] = 0;
      }
    }
    if (done) return -1;
    const double* prev = norm2 + (size_t)((sweep - 1) & 1) * nstride + sw.sig;
    for (int i = tid; i < n; i += blockDim.x) scratch[i] = prev[i];
    if (tid < 2 * JB) vrow[tid] = -1;
    __syncthreads();
    for (int i = tid; i < n; i += blockDim.x) {
      const double v = scratch[i];
      int rank = 0;
      for (int q = 0; q < n; ++q) {
        const double u = scratch[q];
        rank += (u > v) || (u == v && q < i);
      }
      int at = -1;
      if (rank >= vI && rank < vI + nI) at = rank - vI;
      else if (rank >= vJ && rank < vJ + nJ) at = JB + rank - vJ;
      if (at >= 0) {
        vrow[at] = i;
        perm[sw.sig + rank] = i;
      }
    }
  } else if (tid < 2 * JB) {
    const int pos = tid < JB ? vI + tid : vJ + (tid - JB);
    const int lim = tid < JB ? vI + nI : vJ + nJ;
    vrow[tid] = pos < lim ? perm[sw.sig + pos] : -1;
  }
  __syncthreads();
  return nI + nJ;
}

__global__ void __launch_bounds__(256)
jacobi_block_step(const SectorWork* __restrict__ secs, const JacobiPairWork* __restrict__ pairs,
                  int t, int desync, int blocked, int* __restrict__ ctr, double2* __restrict__ theta,
                  double2* __restrict__ accbuf, JacobiOut* __restrict__ st, int* __restrict__ perm,
                  double* __restrict__ norm2, long long nstride, double tol_opt, int max_inner) {
  // xs stages column chunks of the vectors; during the eig it is the second G
  // buffer.  Rows are padded by two elements: with a stride of kJP + 2 the
  // entries one round-robin step reads fall on more distinct LDS banks than
  // with kJP + 1 (whose pair entries (p, q), p + q fixed by the step, share
  // few banks).
  __shared__ double2 xs[kJP][kJP + 2];
  __shared__ double2 gs[kJP][kJP + 2];
  __shared__ double2 ws[kJP][kJP + 2];
  __shared__ double gmax;
  __shared__ int vrow[kJP];
  __shared__ int4 anyf[2];
  int parity = 0;
  const JacobiPairWork w = pairs[blockIdx.x];
  const int sid = w.sector;
  if (st[sid].converged) return;
  const SectorWork sw = secs[sid];
  const bool tall = sw.tall != 0;
  const int n = tall ? sw.c : sw.r;
  const int len = tall ? sw.r : sw.c;
  double2* x = theta + sw.off;
  const double tol = jac_tol(tol_opt, len);
  const double floor_g = (double)len * DBL_EPSILON * DBL_EPSILON * st[sid].fro2;
  const int tid = threadIdx.x;
  // block I holds the vectors at sorted positions 16 I .. 16 I + 15
  int slot = 0, nbuf = 0;
  const int nv = jac_setup<kJB>(w, sw, sid, t, desync, blocked, ctr, st, perm, norm2, nstride,
                                reinterpret_cast<double*>(&xs[0][0]), vrow, slot, nbuf);
  // a block paired with the empty padding block still orthogonalises its own vectors
  if (nv < 2) return;
  bool fresh = false;          // gs holds the Gram matrix of the current vectors
  for (int pass = 0; pass < 2; ++pass) {
    if (!fresh) {
      jac_gram(xs, gs, x, len, vrow);
      if (tid == 0) atomicAdd(&st[sid].gram_units, (unsigned long long)nv * nv * len);
    }
    __syncthreads();
    // ---- largest squared norm (for the coarse noise floor) and any pair
    // above tolerance?  The barrier inside jac_any_above publishes gmax.
    if (tid < 64) {
      double m = tid < kJP ? gs[tid][tid].x : 0.0;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
      if (tid == 0) gmax = m;
    }
    const bool need = jac_any_above(gs, tol, floor_g, anyf, parity);
    if (!need) break;
    if (pass == 0 && tid == 0) atomicAdd(&st[sid].rot3[slot], 1);
    // ---- rotate G (at most max_inner sweeps), W = accumulated product
    for (int e = tid; e < kJP * kJP; e += blockDim.x) {
      const int r = e / kJP, c = e % kJP;
      ws[r][c] = make_double2(r == c ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    const double ptol = pass == 0 ? fmax(tol, kJacLoose) : tol;
    const double pfloor = pass == 0 ? fmax(floor_g, kJacNoise * DBL_EPSILON * gmax) : floor_g;
    if (pass == 0 && !jac_any_above(gs, ptol, pfloor, anyf, parity)) {
      // nothing above the coarse thresholds: gs is still the Gram matrix of
      // the unchanged vectors, go straight to the full-tolerance pass
      fresh = true;
      continue;
    }
    jac_gram_eig(gs, xs, ws, ptol, pfloor, max_inner, anyf, parity);
    // ---- rotate the vectors (and the accumulator of a tall sector)
    jac_apply(xs, ws, x, len, vrow);
    if (tall) jac_apply(xs, ws, accbuf + sw.acc, n, vrow);
    if (tid == 0) atomicAdd(&st[sid].apply_units, (unsigned long long)nv * nv * (len + (tall ? n : 0)));
    fresh = false;
    __syncthreads();
    if (pass == 0) break;
  }
  // latest squared norms of the pair's vectors (the Gram diagonal; after a
  // rotation the rotated Gram's diagonal), for the next sweep's ordering
  __syncthreads();
  if (tid < kJP && vrow[tid] >= 0) norm2[(size_t)nbuf * nstride + sw.sig + vrow[tid]] = gs[tid][tid].x;
}

// ---------------------------------------------------------------------------
// The same visit with blocks of kJB8 = 8 vectors (block pairs of 16).
//
// A 16-vector pair carries a quarter of the Gram and rotation work of a
// 32-vector pair and its eig takes 15 round-robin steps instead of 31, so a
// visit is several times shorter; a sweep has twice the steps and a launch
// twice the workgroups.  The work is laid out for that size: each of the four
// wavefronts takes every fourth 32-column chunk of the vectors through a
// staging tile of its own (no workgroup barrier in the chunk loops), the
// Gram matrix is summed from the four partial products in a fixed order, and
// the eig runs on one wavefront, which owns the whole 16 x 16 problem, with
// the matrices updated in place in LDS (within a wavefront, LDS operations
// complete in issue order, and every read of a step is issued before its
// first write).
constexpr int kJP8 = 2 * kJB8;
constexpr int kJ8Regs = kJP8 * 32 / 64;   // elements of a 16 x 32 chunk per lane
constexpr int kJ8Waves = 4;               // wavefronts per workgroup (8 measured slower)
constexpr int kJ8Threads = 64 * kJ8Waves;

// True (uniform) if pred holds on any thread of the workgroup (flags: two
// alternating sets of per-wavefront words; parity selects the set).
__device__ __forceinline__ bool jac8_block_any(int pred, int (*flags)[kJ8Waves], int& parity) {
  const bool w = __ballot(pred) != 0ull;
  if ((threadIdx.x & 63) == 0) flags[parity][threadIdx.x >> 6] = w ? 1 : 0;
  __syncthreads();
  int v = 0;
#pragma unroll
  for (int i = 0; i < kJ8Waves; ++i) v |= flags[parity][i];
  parity ^= 1;
  return v != 0;
}

// LDS ordering point within one wavefront: the compiler keeps LDS accesses on
// their side, and this lane's LDS operations have completed.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_s_waitcnt(0xc07f);       // lgkmcnt(0), other counters unconstrained
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Pair k of round-robin step s over the 16 rows, (p, q) with p < q (the
// schedule of rr_pair(s, k, 16) with selects instead of divisions).
__device__ __forceinline__ void jac8_pair(int s, int k, int& p, int& q) {
  int i = s + k;
  i = i >= kJP8 - 1 ? i - (kJP8 - 1) : i;
  int j = s - k;
  j = j < 0 ? j + (kJP8 - 1) : j;
  j = k == 0 ? kJP8 - 1 : j;
  p = min(i, j);
  q = max(i, j);
}

// Lane's share of the chunk [c0, c0 + 32) of the 16 rows: element e = lane +
// 64 j is row e / 32, column e % 32, so 32 lanes read one row's 512 bytes.
// rowp[j] is that row's base pointer (null: absent row, reads as 0).
__device__ __forceinline__ void jac8_fetch(double2 (&v)[kJ8Regs], const double2* const (&rowp)[kJ8Regs],
                                           int len, int c0) {
  const int col = c0 + (threadIdx.x & 31);
#pragma unroll
  for (int j = 0; j < kJ8Regs; ++j) {
    v[j] = make_double2(0.0, 0.0);
    if (rowp[j] && col < len) v[j] = rowp[j][col];
  }
}

// Runs body(c0, tile) for the chunks c0 = 32 (w + 4 i) < len of wavefront w,
// each staged in the wavefront's tile; the next chunk's loads are in flight
// while the body works.  The body may overwrite its own chunk's columns.
template <class Body>
__device__ __forceinline__ void jac8_chunks(double2 (*xt)[33], const double2* x, int len, const int* vrow,
                                            Body&& body) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double2* rowp[kJ8Regs];
#pragma unroll
  for (int j = 0; j < kJ8Regs; ++j) {
    const int r = vrow[(lane >> 5) + 2 * j];
    rowp[j] = r >= 0 ? x + (size_t)r * len : nullptr;
  }
  const int nch = (len + 31) >> 5;
  double2 ra[kJ8Regs];
  int ch = wave;
  if (ch < nch) jac8_fetch(ra, rowp, len, ch * 32);
  while (ch < nch) {
    wave_lds_sync();                        // the previous body's tile reads are done
#pragma unroll
    for (int j = 0; j < kJ8Regs; ++j) xt[(lane >> 5) + 2 * j][lane & 31] = ra[j];
    wave_lds_sync();
    const int nx = ch + kJ8Waves;
    if (nx < nch) jac8_fetch(ra, rowp, len, nx * 32);
    body(ch * 32);
    ch = nx;
  }
  wave_lds_sync();
}

// G = X X^H of the 16 rows into gs (exactly Hermitian, from the upper
// triangle).  Each wavefront forms Gr = Xr Xr^T + Xi Xi^T and M = Xi Xr^T over
// its chunks on the matrix cores (lane l supplies X[l % 16][k0 + l / 16] as
// both operands); the partials meet in the staging tiles and are summed in
// wavefront order; Gi = M - M^T.
__device__ void jac8_gram(double2 (*xt)[kJP8][33], double2 (*gs)[kJP8 + 1], const double2* x, int len,
                          const int* vrow) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  double2 (*t)[33] = xt[wave];
  v4d gra = {0.0, 0.0, 0.0, 0.0}, grb = {0.0, 0.0, 0.0, 0.0}, mm = {0.0, 0.0, 0.0, 0.0};
  jac8_chunks(t, x, len, vrow, [&](int) {
#pragma unroll
    for (int k0 = 0; k0 < 32; k0 += 4) {
      const double2 av = t[li][k0 + lk];
      gra = mfma16x16x4(av.x, av.x, gra);
      grb = mfma16x16x4(av.y, av.y, grb);
      mm = mfma16x16x4(av.y, av.x, mm);
    }
  });
  double* part = reinterpret_cast<double*>(&t[0][0]);     // [2][16][16]
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    part[(4 * r + lk) * 16 + li] = gra[r] + grb[r];
    part[256 + (4 * r + lk) * 16 + li] = mm[r];
  }
  __syncthreads();
  {
    const int r = tid >> 4, c = tid & 15;
    if (tid < 256 && r <= c) {
      double gr = 0.0, mrc = 0.0, mcr = 0.0;
#pragma unroll
      for (int w = 0; w < kJ8Waves; ++w) {
        const double* pw = reinterpret_cast<const double*>(&xt[w][0][0]);
        gr += pw[r * 16 + c];
        mrc += pw[256 + r * 16 + c];
        mcr += pw[256 + c * 16 + r];
      }
      const double2 g = make_double2(gr, r == c ? 0.0 : mrc - mcr);
      gs[r][c] = g;
      gs[c][r] = cconj(g);
    }
  }
  __syncthreads();
}

// X <- W X for the 16 rows of a row-major matrix (rows of length len): per
// chunk, two 16 x 16 output tiles, three real products per k-step (Gauss).
__device__ void jac8_apply(double2 (*xt)[kJP8][33], double2 (*ws)[kJP8 + 1], double2* __restrict__ x, int len,
                           const int* vrow) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  double2 (*t)[33] = xt[wave];
  int orow[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) orow[r] = vrow[4 * r + lk];
  jac8_chunks(t, x, len, vrow, [&](int c0) {
#pragma unroll
    for (int jt = 0; jt < 32; jt += 16) {
      v4d p1 = {0.0, 0.0, 0.0, 0.0}, p2 = {0.0, 0.0, 0.0, 0.0}, p3 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int k0 = 0; k0 < kJP8; k0 += 4) {
        const double2 wv = ws[li][k0 + lk];          // A = W[i][k]
        const double2 xv = t[k0 + lk][jt + li];      // B = X[k][jt + j]
        p1 = mfma16x16x4(wv.x, xv.x, p1);
        p2 = mfma16x16x4(wv.y, xv.y, p2);
        p3 = mfma16x16x4(wv.x + wv.y, xv.x + xv.y, p3);
      }
      const int col = c0 + jt + li;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (orow[r] >= 0 && col < len)
          x[(size_t)orow[r] * len + col] = make_double2(p1[r] - p2[r], p3[r] - p1[r] - p2[r]);
    }
  });
}

// True (uniform) if any off-diagonal pair of the 16 x 16 gs is above the
// threshold: thread t checks entry (t / 16, t % 16).
__device__ __forceinline__ bool jac8_any_above(double2 (*gs)[kJP8 + 1], double tol, double floor_g,
                                               int (*anyf)[kJ8Waves], int& parity) {
  const int p = (threadIdx.x >> 4) & 15, q = threadIdx.x & 15;
  const int f = threadIdx.x < 256 && p < q && jac_needs(gs[p][p].x, gs[q][q].x, gs[p][q], tol, floor_g) ? 1 : 0;
  return jac8_block_any(f, anyf, parity);
}

// Rotations of the 16 x 16 gs by wavefront 0, in place: lane 8 A + B owns
// the 2 x 2 blocks (rows of pair A) x (columns of pair B) of G and W, as in
// jac_gram_eig; up to max_inner sweeps of 15 steps.
__device__ void jac8_gram_eig(double2 (*gs)[kJP8 + 1], double2 (*ws)[kJP8 + 1], double tol, double floor_g,
                              int max_inner) {
  const int lane = threadIdx.x & 63;
  const int A = lane >> 3, B = lane & 7;
  for (int inner = 0; inner < max_inner; ++inner) {
    for (int s2 = 0; s2 < kJP8 - 1; ++s2) {
      int pa, qa, pb, qb;
      jac8_pair(s2, A, pa, qa);
      jac8_pair(s2, B, pb, qb);
      const double2 ga = gs[pa][qa], gb = gs[pb][qb];
      const double apa = gs[pa][pa].x, aqa = gs[qa][qa].x, apb = gs[pb][pb].x, aqb = gs[qb][qb].x;
      double2 g00 = gs[pa][pb], g01 = gs[pa][qb], g10 = gs[qa][pb], g11 = gs[qa][qb];
      double2 w00 = ws[pa][pb], w01 = ws[pa][qb], w10 = ws[qa][pb], w11 = ws[qa][qb];
      double ca, wra, wia, cb, wrb, wib;
      jac_rotation(apa, aqa, ga.x, ga.y, tol, floor_g, ca, wra, wia);
      jac_rotation(apb, aqb, gb.x, gb.y, tol, floor_g, cb, wrb, wib);
      rot_pair(g00, g10, ca, wra, wia);
      rot_pair(g01, g11, ca, wra, wia);
      rot_pair(w00, w10, ca, wra, wia);
      rot_pair(w01, w11, ca, wra, wia);
      rot_pair(g00, g01, cb, wrb, -wib);
      rot_pair(g10, g11, cb, wrb, -wib);
      // every read of this step is issued before the first write
      wave_lds_sync();
      ws[pa][pb] = w00; ws[pa][qb] = w01; ws[qa][pb] = w10; ws[qa][qb] = w11;
      gs[pa][pb] = g00; gs[pa][qb] = g01; gs[qa][pb] = g10; gs[qa][qb] = g11;
      wave_lds_sync();
    }
    if (inner + 1 < max_inner) {
      int f = 0;
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int p = 2 * A + i, q = 2 * B + j;
          if (p < q && jac_needs(gs[p][p].x, gs[q][q].x, gs[p][q], tol, floor_g)) f = 1;
        }
      if (__ballot(f) == 0ull) break;
    }
  }
}

// One round-robin step over blocks of 8 for every active sector: one
// workgroup of 256 threads per block pair.  Visit rule, thresholds and
// bookkeeping as in jacobi_block_step.
__global__ void __launch_bounds__(kJ8Threads)
jacobi_block_step8(const SectorWork* __restrict__ secs, const JacobiPairWork* __restrict__ pairs,
                   int t, int desync, int blocked, int* __restrict__ ctr, double2* __restrict__ theta,
                   double2* __restrict__ accbuf, JacobiOut* __restrict__ st, int* __restrict__ perm,
                   double* __restrict__ norm2, long long nstride, double tol_opt, int max_inner) {
  __shared__ double2 xt[kJ8Waves][kJP8][33];
  __shared__ double2 gs[kJP8][kJP8 + 1];
  __shared__ double2 ws[kJP8][kJP8 + 1];
  __shared__ double gmax;
  __shared__ int vrow[kJP8];
  __shared__ int anyf[2][kJ8Waves];
  int parity = 0;
  const JacobiPairWork w = pairs[blockIdx.x];
  const int sid = w.sector;
  if (st[sid].converged) return;
  const SectorWork sw = secs[sid];
  const bool tall = sw.tall != 0;
  const int n = tall ? sw.c : sw.r;
  const int len = tall ? sw.r : sw.c;
  double2* x = theta + sw.off;
  const double tol = jac_tol(tol_opt, len);
  const double floor_g = (double)len * DBL_EPSILON * DBL_EPSILON * st[sid].fro2;
  const int tid = threadIdx.x;
  int slot = 0, nbuf = 0;
  const int nv = jac_setup<kJB8>(w, sw, sid, t, desync, blocked, ctr, st, perm, norm2, nstride,
                                 reinterpret_cast<double*>(&xt[0][0][0]), vrow, slot, nbuf);
  if (nv < 2) return;
  bool fresh = false;
  for (int pass = 0; pass < 2; ++pass) {
    if (!fresh) {
      jac8_gram(xt, gs, x, len, vrow);
      if (tid == 0) atomicAdd(&st[sid].gram_units, (unsigned long long)nv * nv * len);
    }
    if (tid < 64) {
      double m = tid < kJP8 ? gs[tid][tid].x : 0.0;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
      if (tid == 0) gmax = m;
    }
    const bool need = jac8_any_above(gs, tol, floor_g, anyf, parity);
    if (!need) break;
    if (pass == 0 && tid == 0) atomicAdd(&st[sid].rot3[slot], 1);
    if (tid < 256) {
      const int r = tid >> 4, c = tid & 15;
      ws[r][c] = make_double2(r == c ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    const double ptol = pass == 0 ? fmax(tol, kJacLoose) : tol;
    const double pfloor = pass == 0 ? fmax(floor_g, kJacNoise * DBL_EPSILON * gmax) : floor_g;
    if (pass == 0 && !jac8_any_above(gs, ptol, pfloor, anyf, parity)) {
      fresh = true;
      continue;
    }
    if (tid < 64) jac8_gram_eig(gs, ws, ptol, pfloor, max_inner);
    __syncthreads();
    jac8_apply(xt, ws, x, len, vrow);
    if (tall) jac8_apply(xt, ws, accbuf + sw.acc, n, vrow);
    if (tid == 0) atomicAdd(&st[sid].apply_units, (unsigned long long)nv * nv * (len + (tall ? n : 0)));
    fresh = false;
    __syncthreads();
    if (pass == 0) break;
  }
  __syncthreads();
  if (tid < kJP8 && vrow[tid] >= 0) norm2[(size_t)nbuf * nstride + sw.sig + vrow[tid]] = gs[tid][tid].x;
}

// Scalar one-sided Jacobi sweeps on the vectors themselves, for the rare
// sector the blocked sweeps leave unconverged.  One workgroup per listed
// sector; each wavefront takes whole vector pairs of a round-robin step,
// forms alpha, beta, gamma with wave reductions and rotates both vectors (and
// the accumulator rows of a tall sector).  A 2x2 rotation has only two-term
// rounding, so it reaches cosines of order sqrt(len) eps, well inside the
// tolerance.  Runs up to max_sweeps sweeps and marks the sector converged
// when a sweep rotates nothing.
__global__ void __launch_bounds__(256)
jacobi_polish(const SectorWork* __restrict__ secs, const int* __restrict__ list,
              double2* __restrict__ theta, double2* __restrict__ accbuf,
              JacobiOut* __restrict__ st, double tol_opt, int max_sweeps) {
  __shared__ int rotated;
  const int sid = list[blockIdx.x];
  if (st[sid].converged) return;
  const SectorWork sw = secs[sid];
  const bool tall = sw.tall != 0;
  const int n = tall ? sw.c : sw.r;
  const int len = tall ? sw.r : sw.c;
  double2* x = theta + sw.off;
  double2* acc = tall ? accbuf + sw.acc : nullptr;
  const double tol = jac_tol(tol_opt, len);
  const double floor_g = (double)len * DBL_EPSILON * DBL_EPSILON * st[sid].fro2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const int np = n + (n & 1);
  bool converged = false;
  int sweeps = 0;
  for (int sweep = 0; sweep < max_sweeps && !converged; ++sweep) {
    __syncthreads();
    if (threadIdx.x == 0) rotated = 0;
    __syncthreads();
    for (int step = 0; step < np - 1; ++step) {
      for (int k = wave; k < np / 2; k += nwaves) {
        int i, j;
        rr_pair(step, k, np, i, j);
        if (i >= n || j >= n) continue;
        double2* xi = x + (size_t)i * len;
        double2* xj = x + (size_t)j * len;
        double al = 0.0, be = 0.0, gr = 0.0, gi = 0.0;
        for (int col = lane; col < len; col += 64) {
          const double2 a = xi[col], b = xj[col];
          al = fma(a.x, a.x, fma(a.y, a.y, al));
          be = fma(b.x, b.x, fma(b.y, b.y, be));
          gr = fma(a.x, b.x, fma(a.y, b.y, gr));
          gi = fma(a.y, b.x, fma(-a.x, b.y, gi));
        }
        al = wave_sum(al); be = wave_sum(be); gr = wave_sum(gr); gi = wave_sum(gi);
        double c, wr, wi;
        if (!jac_rotation(al, be, gr, gi, tol, floor_g, c, wr, wi)) continue;
        for (int col = lane; col < len; col += 64) {
          double2 a = xi[col], b = xj[col];
          rot_pair(a, b, c, wr, wi);
          xi[col] = a;
          xj[col] = b;
        }
        if (tall) {
          double2* ai = acc + (size_t)i * n;
          double2* aj = acc + (size_t)j * n;
          for (int col = lane; col < n; col += 64) {
            double2 a = ai[col], b = aj[col];
            rot_pair(a, b, c, wr, wi);
            ai[col] = a;
            aj[col] = b;
          }
        }
        if (lane == 0) rotated = 1;
      }
      __syncthreads();
    }
    ++sweeps;
    converged = rotated == 0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    st[sid].sweeps += sweeps;
    st[sid].converged = converged ? 1 : 0;
  }
}

// After a sweep: a sector with no rotated block pair is converged.  One
// workgroup; *active receives 1 if any sector still rotates.
__global__ void __launch_bounds__(1024)
jacobi_sweep_end(const int* __restrict__ list, const int* __restrict__ nbs, int count, JacobiOut* __restrict__ st,
                 int* __restrict__ active) {
  __shared__ int act, maxnb;
  if (threadIdx.x == 0) {
    act = 0;
    maxnb = 0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < count; i += blockDim.x) {
    const int s = list[i];
    JacobiOut o = st[s];
    if (o.converged) continue;
    o.sweeps += 1;
    o.rotations += o.rot3[0];
    if (o.rot3[0] == 0) {
      o.converged = 1;
    } else {
      atomicOr(&act, 1);
      atomicMax(&maxnb, nbs[i]);
    }
    o.rot3[0] = 0;
    st[s] = o;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    active[0] = act;
    active[1] = maxnb;
  }
}

// Between sweeps: order every still-active sector's vectors by descending
// norm (ties: lower index first), so that blocks hold vectors of similar
// size.  One workgroup per sector; the norms are compared from LDS (n
// doubles of dynamic shared memory).
__global__ void __launch_bounds__(256)
jacobi_sort(const SectorWork* __restrict__ secs, const int* __restrict__ list,
            const JacobiOut* __restrict__ st, int* __restrict__ perm,
            const double* __restrict__ norm2) {
  extern __shared__ double jsv[];
  const int sid = list[blockIdx.x];
  if (st[sid].converged) return;
  const SectorWork sw = secs[sid];
  const int n = sw.tall ? sw.c : sw.r;
  const double* nv = norm2 + sw.sig;
  for (int i = threadIdx.x; i < n; i += blockDim.x) jsv[i] = nv[i];
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double v = jsv[i];
    int rank = 0;
    for (int k = 0; k < n; ++k) {
      const double w = jsv[k];
      rank += (w > v) || (w == v && k < i);
    }
    perm[sw.sig + rank] = i;
  }
}

// One workgroup of kJacRowThreads per sector: vector norms -> singular
// values (a wavefront per vector), V^dagger rows into the sector's slot
// (stride c), order by descending value.
__global__ void __launch_bounds__(kJacRowThreads)
jacobi_finalize(const SectorWork* __restrict__ secs, const int* __restrict__ list,
                double2* __restrict__ theta, const double2* __restrict__ accbuf,
                double* __restrict__ sigma, int* __restrict__ order) {
  extern __shared__ double jsm[];          // n doubles
  const int sid = list[blockIdx.x];
  const SectorWork sw = secs[sid];
  const bool tall = sw.tall != 0;
  const int n = tall ? sw.c : sw.r;
  const int len = tall ? sw.r : sw.c;
  double2* x = theta + sw.off;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  for (int i = wave; i < n; i += nwaves) {
    double2* xi = x + (size_t)i * len;
    double ss = 0.0;
    for (int col = lane; col < len; col += 64) {
      const double2 a = xi[col];
      ss = fma(a.x, a.x, fma(a.y, a.y, ss));
    }
    ss = wave_sum(ss);
    const double nr = sqrt(ss);
    if (!tall && nr > 0.0) {
      const double inv = 1.0 / nr;
      for (int col = lane; col < len; col += 64) {
        const double2 a = xi[col];
        xi[col] = make_double2(a.x * inv, a.y * inv);
      }
    }
    if (lane == 0) jsm[i] = nr;
  }
  __syncthreads();
  if (tall) {
    const double2* a = accbuf + sw.acc;
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) x[e] = cconj(a[e]);
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double v = jsm[i];
    int rank = 0;
    for (int k = 0; k < n; ++k) {
      const double w = jsm[k];
      rank += (w > v) || (w == v && k < i);
    }
    sigma[sw.sig + rank] = v;
    order[sw.sig + rank] = i;
  }
}


// ---------------------------------------------------------------------------
// Host launchers.

hipError_t launch_jacobi_init(const SectorWork* secs, const int* list, int count,
                              const double2* theta, double2* acc, JacobiOut* st, int* perm,
                              double* norm2, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(jacobi_init, dim3(count), dim3(kJacRowThreads), 0, s, secs, list, theta, acc, st, perm, norm2);
  return hipGetLastError();
}

hipError_t launch_jacobi_sort(const SectorWork* secs, const int* list, int count, int maxrows, const JacobiOut* st,
                              int* perm, const double* norm2, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const size_t smem = (size_t)maxrows * sizeof(double);
  hipLaunchKernelGGL(jacobi_sort, dim3(count), dim3(256), smem, s, secs, list, st, perm, norm2);
  return hipGetLastError();
}

int jacobi_desync_rows(int block) {
  return block == kJB8 ? kJ8Waves * kJP8 * 33 * 2 : kJP * (kJP + 2) * 2;
}

hipError_t launch_jacobi_step(const SectorWork* secs, const JacobiPairWork* pairs, int npairs, int t,
                              int desync, int blocked, int* ctr, double2* theta, double2* acc, JacobiOut* st,
                              int* perm, double* norm2, long long nstride, double tol, int max_inner, int block,
                              hipStream_t s) {
  if (npairs <= 0) return hipSuccess;
  if (block == kJB8)
    hipLaunchKernelGGL(jacobi_block_step8, dim3(npairs), dim3(kJ8Threads), 0, s, secs, pairs, t, desync, blocked,
                       ctr, theta, acc, st, perm, norm2, nstride, tol, max_inner);
  else if (block == kJB)
    hipLaunchKernelGGL(jacobi_block_step, dim3(npairs), dim3(256), 0, s, secs, pairs, t, desync, blocked, ctr,
                       theta, acc, st, perm, norm2, nstride, tol, max_inner);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_jacobi_sweep_end(const int* list, const int* nbs, int count, JacobiOut* st, int* active,
                                   hipStream_t s) {
  hipLaunchKernelGGL(jacobi_sweep_end, dim3(1), dim3(1024), 0, s, list, nbs, count, st, active);
  return hipGetLastError();
}

hipError_t launch_jacobi_polish(const SectorWork* secs, const int* list, int count, double2* theta,
                                double2* acc, JacobiOut* st, double tol, int max_sweeps, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(jacobi_polish, dim3(count), dim3(256), 0, s, secs, list, theta, acc, st, tol, max_sweeps);
  return hipGetLastError();
}

hipError_t launch_jacobi_finalize(const SectorWork* secs, const int* list, int count, int maxrows,
                                  double2* theta, const double2* acc, double* sigma, int* order,
                                  hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const size_t smem = (size_t)maxrows * sizeof(double);
  hipLaunchKernelGGL(jacobi_finalize, dim3(count), dim3(kJacRowThreads), smem, s, secs, list, theta, acc, sigma,
                     order);
  return hipGetLastError();
}

}  // namespace u1mps
