// gfx950 kernels of the U(1)-symmetric MPS two-site update and read-outs.
//
// Steps of one update on sites (s, s+1) (Sec. II of arXiv 2303.11409):
//   theta_kernel   Theta~(cL, m, cR) = sum_cM G^(n)[(cL-m), (cL-cM)] B[s](cL,cM) B[s+1](cM,cR)
//                  (charge-sector-matched products, gate mixed per n = cL - cR
//                  in the epilogue), plus Theta = lambda_s * Theta~ for the SVD.
//   jacobi_rows    one-sided (Hestenes) Jacobi on the rows of every Theta(m):
//                  rotations until all row pairs are orthogonal; the row norms
//                  are the singular values and the normalised rows are V^dagger.
//   select_kernel  one cut over all sectors of a gate: sort, discarded-weight
//                  rule, chi cap, kept count per sector (FP64).
//   update_*       new B[s+1] = kept V^dagger rows, lambda = kept values,
//                  new B[s] = Theta~ V_kept (generic complex GEMM).
// Wave64 throughout: reductions use cross-lane shuffles over 64 lanes.
#include "kernels.h"

#include <float.h>
#include <math.h>

namespace u1mps {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ void cfma(double2& acc, double2 a, double2 b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// FP64 matrix-core product D[16x16] += A[16x4] B[4x16] on one wavefront.
// Lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; register r of lane
// l holds D[4 r + l / 16][l % 16].
typedef double v4d __attribute__((ext_vector_type(4)));
__device__ __forceinline__ v4d mfma16x16x4(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Theta formation.  One workgroup (256 threads, 16 x 16) per 32 x 32 tile of
// one (cL, cR) pair; each thread owns rows ty, ty+16 and columns tx, tx+16.
template <int W>
__global__ void __launch_bounds__(256)
theta_kernel(const GateWork* __restrict__ gates, const ThetaTile* __restrict__ tiles,
             const SectorWork* __restrict__ secs, const double2* __restrict__ coef,
             double2* __restrict__ th_raw, double2* __restrict__ th_scaled) {
  __shared__ ThetaTile t;
  __shared__ double2 as[kThetaTile][17];
  __shared__ double2 bs[16][kThetaTile + 1];
  if (threadIdx.x == 0) t = tiles[blockIdx.x];
  __syncthreads();
  const GateWork g = gates[t.gate];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;

  double2 out[W][2][2];
#pragma unroll
  for (int i = 0; i < W; ++i)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) out[i][a][b] = make_double2(0.0, 0.0);

  for (int j = 0; j < t.nin; ++j) {
    double2 p[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) p[a][b] = make_double2(0.0, 0.0);
    const int kb = t.k0[j], ke = t.k0[j] + t.kn[j];
    for (int k0 = kb; k0 < ke; k0 += 16) {
      // A tile: 32 rows x 16 k, two elements per thread
      for (int e = threadIdx.x; e < kThetaTile * 16; e += 256) {
        const int r = e >> 4, kk = e & 15;
        const int k = k0 + kk;
        double2 v = make_double2(0.0, 0.0);
        if (r < t.nrow && k < ke) v = g.bl[(size_t)(t.row0 + r) * g.ldl + k];
        as[r][kk] = v;
      }
      // B tile: 16 k x 32 columns
      for (int e = threadIdx.x; e < 16 * kThetaTile; e += 256) {
        const int kk = e >> 5, c = e & 31;
        const int k = k0 + kk;
        double2 v = make_double2(0.0, 0.0);
        if (c < t.ncol && k < ke) v = g.br[(size_t)k * g.ldr + t.col0 + c];
        bs[kk][c] = v;
      }
      __syncthreads();
#pragma unroll 4
      for (int kk = 0; kk < 16; ++kk) {
        const double2 a0 = as[ty][kk], a1 = as[ty + 16][kk];
        const double2 b0 = bs[kk][tx], b1 = bs[kk][tx + 16];
        cfma(p[0][0], a0, b0);
        cfma(p[0][1], a0, b1);
        cfma(p[1][0], a1, b0);
        cfma(p[1][1], a1, b1);
      }
      __syncthreads();
    }
    // gate mix: out_i += G^(n)[p_i][a_j] * P_j
#pragma unroll
    for (int i = 0; i < W; ++i) {
      if (i < t.nout) {
        const double2 gc = coef[g.coef + (t.n * g.d + t.p[i]) * g.d + t.a[j]];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) cfma(out[i][a][b], gc, p[a][b]);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < W; ++i) {
    if (i < t.nout) {
      const SectorWork s = secs[t.sec[i]];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int r = ty + 16 * a;
        if (r >= t.nrow) continue;
        const double lam = g.lam_l[t.row0 + r];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int c = tx + 16 * b;
          if (c >= t.ncol) continue;
          const size_t rr = (size_t)(t.orow[i] + r), cc = (size_t)(t.ocol[i] + c);
          const double2 v = out[i][a][b];
          th_raw[(size_t)s.off + rr * s.c + cc] = v;
          // the SVD input of a tall sector is stored transposed (its columns as rows)
          const size_t si = s.tall ? (size_t)s.off + cc * s.r + rr : (size_t)s.off + rr * s.c + cc;
          th_scaled[si] = make_double2(lam * v.x, lam * v.y);
        }
      }
    }
  }
}

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
// matrix G = X X^H of its 2 kJB vectors, applies the same rotations to G
// (G <- U G U^H) until its off-diagonal is below tolerance, accumulating
// W = prod U, and finally rotates the vectors, X <- W X.  Convergence is
// always judged on a Gram matrix freshly formed from the vectors, so the
// stopping rule is the same pairwise-cosine test as for the unblocked method.
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
  if (!(g2 > tol * tol * al * be) || !(g2 > floor_g * floor_g)) return false;
  // with delta = beta - alpha, r = sqrt(delta^2 + 4|gamma|^2), D = |delta| + r:
  // c = D / E, w = 2 sgn(delta) gamma / E with E^2 = D^2 + 4|gamma|^2 = 2 r D --
  // the same rotation as t = sgn(zeta) / (|zeta| + sqrt(1 + zeta^2)),
  // zeta = delta / (2|gamma|), c = 1/sqrt(1 + t^2), w = c t gamma/|gamma|
  const double delta = be - al;
  const double r = sqrt(delta * delta + 4.0 * g2);
  const double D = fabs(delta) + r;
  const double inv = rsqrt(2.0 * r * D);
  const double sg = delta >= 0.0 ? 2.0 * inv : -2.0 * inv;
  c = D * inv;
  wr = sg * gr;
  wi = sg * gi;
  return true;
}

// Default threshold: (vector length) * eps, but never below 2 * kJP * eps,
// the rounding level of the kJP-term combinations X <- W X that rotate a
// block pair (short vectors would otherwise be held to a test they cannot
// pass).
__device__ __forceinline__ double jac_tol(double tol_opt, int len) {
  return tol_opt > 0.0 ? tol_opt : (double)max(len, 2 * kJP) * DBL_EPSILON;
}

// One workgroup per sector: reset state, vector norms, identity order,
// squared Frobenius norm, A = I.
__global__ void __launch_bounds__(256)
jacobi_init(const SectorWork* __restrict__ secs, const int* __restrict__ list,
            const double2* __restrict__ theta, double2* __restrict__ accbuf,
            JacobiOut* __restrict__ st, int* __restrict__ perm, double* __restrict__ norm2) {
  __shared__ double wsum[4];
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
  for (int i = wave; i < n; i += 4) {
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
    o.rot_this_sweep = 0;
    o.gram_units = 0;
    o.apply_units = 0;
    o.fro2 = wsum[0] + wsum[1] + wsum[2] + wsum[3];
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

__device__ __forceinline__ void jac_stage(double2 (*xs)[33], const double2 (&v)[kJChunkRegs]) {
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
__device__ __forceinline__ void jac_chunk_loop(double2 (*xs)[33], const double2* x, int len,
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
// quadrant (rows 16 (w / 2), columns 16 (w % 2)) of each chunk as four real
// products per k-step, Or = Wr Xr - Wi Xi and Oi = Wr Xi + Wi Xr.
__device__ void jac_apply(double2 (*xs)[33], double2 (*ws)[kJP + 1], double2* __restrict__ x,
                          int len, const int* vrow) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int R = (wave >> 1) * 16, Cq = (wave & 1) * 16;
  const int li = lane & 15, lk = lane >> 4;
  jac_chunk_loop(xs, x, len, vrow, [&](int c0) {
    v4d orr = {0.0, 0.0, 0.0, 0.0}, oi = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k0 = 0; k0 < kJP; k0 += 4) {
      const double2 wv = ws[R + li][k0 + lk];      // A = W[R + i][k]
      const double2 xv = xs[k0 + lk][Cq + li];     // B = X[k][C + j]
      orr = mfma16x16x4(wv.x, xv.x, orr);
      orr = mfma16x16x4(-wv.y, xv.y, orr);
      oi = mfma16x16x4(wv.x, xv.y, oi);
      oi = mfma16x16x4(wv.y, xv.x, oi);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int v = vrow[R + 4 * r + lk];
      const int col = c0 + Cq + li;
      if (v >= 0 && col < len) x[(size_t)v * len + col] = make_double2(orr[r], oi[r]);
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
__device__ void jac_gram(double2 (*xs)[33], double2 (*gs)[kJP + 1], const double2* x, int len,
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
__device__ __forceinline__ bool jac_any_above(double2 (*gs)[kJP + 1], double tol, double floor_g,
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

// Rotations of the Gram matrix gs (in LDS) until no pair exceeds the
// threshold; W accumulates the product.  The caller has established that
// some pair is above it.  A round-robin step rotates 16 disjoint pairs at
// once, G <- U G U^H and W <- U W with U block diagonal over the pairs: 16
// threads compute the pairs' rotations into rot[], then thread t = 16 A + B
// updates the 2 x 2 blocks (rows of pair A) x (columns of pair B) of G and W
// in place (each block is read and written by its owner only).  After each
// sweep one parallel test over all pairs replaces the sweep that would find
// nothing to rotate (it would leave G and W unchanged).
__device__ void jac_gram_eig(double2 (*gs)[kJP + 1], double2 (*ws)[kJP + 1], double4* rot,
                             double tol, double floor_g, int max_inner, int4* anyf, int& parity) {
  const int tid = threadIdx.x;
  const int A = tid >> 4, B = tid & 15;
  for (int inner = 0; inner < max_inner; ++inner) {
    for (int s2 = 0; s2 < kJP - 1; ++s2) {
      // G and W change only in update phases, each closed by a barrier, so
      // this thread's block is read before the rotations are published
      int pa, qa, pb, qb;
      jac_pair_fast(s2, A, pa, qa);
      jac_pair_fast(s2, B, pb, qb);
      double2 g00 = gs[pa][pb], g01 = gs[pa][qb], g10 = gs[qa][pb], g11 = gs[qa][qb];
      double2 w00 = ws[pa][pb], w01 = ws[pa][qb], w10 = ws[qa][pb], w11 = ws[qa][qb];
      int flag = 0;
      if (tid < kJP / 2) {
        int p, q;
        jac_pair_fast(s2, tid, p, q);
        double c = 1.0, wr = 0.0, wi = 0.0;
        const double2 g = gs[p][q];
        flag = jac_rotation(gs[p][p].x, gs[q][q].x, g.x, g.y, tol, floor_g, c, wr, wi) ? 1 : 0;
        rot[tid] = make_double4(c, wr, wi, flag ? 1.0 : 0.0);
      }
      if (!block_any(flag, anyf, parity)) continue;
      const double4 ra = rot[A], rb = rot[B];
      if (ra.w != 0.0 || rb.w != 0.0) {
        if (ra.w != 0.0) {        // rows pa, qa: U from the left, also on W
          rot_pair(g00, g10, ra.x, ra.y, ra.z);
          rot_pair(g01, g11, ra.x, ra.y, ra.z);
          rot_pair(w00, w10, ra.x, ra.y, ra.z);
          rot_pair(w01, w11, ra.x, ra.y, ra.z);
          ws[pa][pb] = w00; ws[pa][qb] = w01; ws[qa][pb] = w10; ws[qa][qb] = w11;
        }
        if (rb.w != 0.0) {        // columns pb, qb: U^H from the right
          rot_pair(g00, g01, rb.x, rb.y, -rb.z);
          rot_pair(g10, g11, rb.x, rb.y, -rb.z);
        }
        gs[pa][pb] = g00; gs[pa][qb] = g01; gs[qa][pb] = g10; gs[qa][qb] = g11;
      }
      __syncthreads();
    }
    if (!jac_any_above(gs, tol, floor_g, anyf, parity)) break;
  }
  __syncthreads();
}

// One round-robin step for every active sector: one workgroup per block pair.
//
// A block pair that fails the convergence test is rotated in two passes.
// Pass 0 diagonalises its Gram matrix only down to kJacLoose relative
// off-diagonal or the Gram's own rounding level (kJacNoise * eps * max
// diagonal): rotations of G itself carry errors of order eps * max|G|, which
// would leave the smallest vectors of the pair with cosines of
// eps * s_max^2 / (s_p s_q) if pursued further.  Pass 1 forms the Gram matrix
// afresh from the rotated vectors; it is then nearly diagonal, its rotations
// are small, their errors are relative to each vector's own norm, and it is
// driven to the full tolerance.
constexpr double kJacLoose = 1e-8;
constexpr double kJacNoise = 64.0;

__global__ void __launch_bounds__(256)
jacobi_block_step(const SectorWork* __restrict__ secs, const JacobiBlockWork* __restrict__ jb,
                  int njb, int step, double2* __restrict__ theta, double2* __restrict__ accbuf,
                  JacobiOut* __restrict__ st, const int* __restrict__ perm, double* __restrict__ norm2,
                  double tol_opt, int max_inner) {
  __shared__ double2 xs[kJP][33];
  __shared__ double2 gs[kJP][kJP + 1];
  __shared__ double2 ws[kJP][kJP + 1];
  __shared__ double gmax;
  __shared__ int vrow[kJP];
  __shared__ double4 rot[kJP / 2];
  __shared__ int4 anyf[2];
  int parity = 0;
  int lo = 0, hi = njb - 1;
  const int pid = blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jb[mid].pair_begin <= pid) lo = mid; else hi = mid - 1;
  }
  const JacobiBlockWork w = jb[lo];
  if (step >= w.nb - 1) return;
  const int sid = w.sector;
  if (st[sid].converged) return;
  const SectorWork sw = secs[sid];
  const bool tall = sw.tall != 0;
  const int n = tall ? sw.c : sw.r;
  const int len = tall ? sw.r : sw.c;
  double2* x = theta + sw.off;
  const double tol = jac_tol(tol_opt, len);
  const double floor_g = (double)len * DBL_EPSILON * DBL_EPSILON * st[sid].fro2;
  int bi, bj;
  rr_pair(step, pid - w.pair_begin, w.nb, bi, bj);
  const int vI = bi * kJB, vJ = bj * kJB;
  const int nI = max(0, min(kJB, n - vI)), nJ = max(0, min(kJB, n - vJ));
  const int nv = nI + nJ;
  const int tid = threadIdx.x;
  // a block paired with the empty padding block still orthogonalises its own vectors
  if (nv < 2) return;
  // block I holds the vectors at sorted positions 16 I .. 16 I + 15
  if (tid < kJP) {
    const int pos = tid < kJB ? vI + tid : vJ + (tid - kJB);
    const int lim = tid < kJB ? vI + nI : vJ + nJ;
    vrow[tid] = pos < lim ? perm[sw.sig + pos] : -1;
  }
  __syncthreads();
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
    if (pass == 0 && tid == 0) atomicAdd(&st[sid].rot_this_sweep, 1);
    // ---- diagonalise G by rotations, W = accumulated product
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
    jac_gram_eig(gs, ws, rot, ptol, pfloor, max_inner, anyf, parity);
    // ---- rotate the vectors (and the accumulator of a tall sector)
    jac_apply(xs, ws, x, len, vrow);
    if (tall) jac_apply(xs, ws, accbuf + sw.acc, n, vrow);
    if (tid == 0) atomicAdd(&st[sid].apply_units, (unsigned long long)nv * nv * (len + (tall ? n : 0)));
    fresh = false;
    __syncthreads();
  }
  // latest squared norms of the pair's vectors (the Gram diagonal; after a
  // rotation the rotated Gram's diagonal), for the next sweep's ordering
  __syncthreads();
  if (tid < kJP && vrow[tid] >= 0) norm2[sw.sig + vrow[tid]] = gs[tid][tid].x;
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
jacobi_sweep_end(const int* __restrict__ list, int count, JacobiOut* __restrict__ st,
                 int* __restrict__ active) {
  __shared__ int act;
  if (threadIdx.x == 0) act = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < count; i += blockDim.x) {
    const int s = list[i];
    JacobiOut o = st[s];
    if (o.converged) continue;
    o.sweeps += 1;
    o.rotations += o.rot_this_sweep;
    if (o.rot_this_sweep == 0) o.converged = 1;
    else atomicOr(&act, 1);
    o.rot_this_sweep = 0;
    st[s] = o;
  }
  __syncthreads();
  if (threadIdx.x == 0) *active = act;
}

// Between sweeps: order every still-active sector's vectors by descending
// norm (ties: lower index first), so that blocks hold vectors of similar
// size.  One workgroup per sector.
__global__ void __launch_bounds__(256)
jacobi_sort(const SectorWork* __restrict__ secs, const int* __restrict__ list,
            const JacobiOut* __restrict__ st, int* __restrict__ perm,
            const double* __restrict__ norm2) {
  const int sid = list[blockIdx.x];
  if (st[sid].converged) return;
  const SectorWork sw = secs[sid];
  const int n = sw.tall ? sw.c : sw.r;
  const double* nv = norm2 + sw.sig;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double v = nv[i];
    int rank = 0;
    for (int k = 0; k < n; ++k) {
      const double w = nv[k];
      rank += (w > v) || (w == v && k < i);
    }
    perm[sw.sig + rank] = i;
  }
}

// One workgroup per sector: vector norms -> singular values, V^dagger rows
// into the sector's slot (stride c), order by descending value.
__global__ void __launch_bounds__(256)
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
// Cut over all sectors of one gate.  One workgroup per gate.  Entries are
// (value, key) with key = local sector << 20 | rank; they are sorted by value
// descending, then key ascending (bitonic network), and the kept count is
//   K = max(1, min(K_eps, K_zero, chi_max, keep_cap, T)).
__device__ __forceinline__ bool sel_before(double va, int ka, double vb, int kb) {
  return va > vb || (va == vb && ka < kb);
}

__global__ void __launch_bounds__(1024)
select_kernel(const GateWork* __restrict__ gates, const SectorWork* __restrict__ secs,
              const double* __restrict__ sigma, double* __restrict__ gsv, int* __restrict__ gsk,
              const long long* __restrict__ scratch_off, int* __restrict__ kept,
              CutOut* __restrict__ cut, int lds_cap) {
  extern __shared__ double ssm[];
  __shared__ int cnt[1024];
  __shared__ double chunk[1024];
  __shared__ int kmin, kzero, nf_flag;
  __shared__ double disc_sh;
  __shared__ int total_sh;
  const int gi = blockIdx.x;
  const GateWork g = gates[gi];
  const int nsec = g.sec_end - g.sec_begin;
  const int tid = threadIdx.x, nt = blockDim.x;

  // total number of candidate values
  if (tid == 0) {
    int t = 0;
    for (int s = g.sec_begin; s < g.sec_end; ++s) t += secs[s].kmax;
    total_sh = t;
  }
  for (int s = tid; s < nsec && s < 1024; s += nt) cnt[s] = 0;
  __syncthreads();
  const int T = total_sh;
  int P = 1;
  while (P < T) P <<= 1;
  double* sv;
  int* sk;
  if (P <= lds_cap) {
    sv = ssm;
    sk = reinterpret_cast<int*>(ssm + P);
  } else {
    sv = gsv + scratch_off[gi];
    sk = gsk + scratch_off[gi];
  }
  // gather
  for (int i = tid; i < P; i += nt) {
    sv[i] = -1.0;
    sk[i] = 0x7fffffff;
  }
  __syncthreads();
  {
    // each sector's first kmax values, sector by sector
    int base = 0;
    for (int s = g.sec_begin; s < g.sec_end; ++s) {
      const SectorWork w = secs[s];
      for (int j = tid; j < w.kmax; j += nt) {
        sv[base + j] = sigma[w.sig + j];
        sk[base + j] = ((s - g.sec_begin) << 20) | j;
      }
      base += w.kmax;
    }
  }
  __syncthreads();
  // bitonic sort, best first
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = tid; i < P; i += nt) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const double va = sv[i], vb = sv[ixj];
          const int ka = sk[i], kb = sk[ixj];
          const bool up = (i & k) == 0;
          const bool sw = up ? sel_before(vb, kb, va, ka) : sel_before(va, ka, vb, kb);
          if (sw) {
            sv[i] = vb; sv[ixj] = va;
            sk[i] = kb; sk[ixj] = ka;
          }
        }
      }
      __syncthreads();
    }
  }
  const double s0 = sv[0];
  bool bad = !(s0 > 0.0) || !isfinite(s0);
  // chunked sums of squares over the T valid entries, in sorted order
  const int C = (T + nt - 1) / nt;
  const int cb = tid * C, ce = min(T, cb + C);
  double part = 0.0;
  int nonfinite = 0;
  for (int i = cb; i < ce; ++i) {
    const double v = sv[i];
    if (!isfinite(v)) nonfinite = 1;
    part = fma(v, v, part);
  }
  chunk[tid] = part;
  if (tid == 0) { kmin = T; kzero = 0; nf_flag = 0; disc_sh = 0.0; }
  __syncthreads();
  if (nonfinite) atomicOr(&nf_flag, 1);
  __syncthreads();
  if (nf_flag) bad = true;
  if (tid == 0) {
    // suffix sums of the chunk sums, fixed order
    double run = 0.0;
    for (int t = nt - 1; t >= 0; --t) {
      const double v = chunk[t];
      chunk[t] = run;          // sum of chunks after t
      run += v;
    }
    disc_sh = run;             // temporarily: total weight W
  }
  __syncthreads();
  const double W = disc_sh;
  const double thr = g.cutoff * W;
  const double zthr = g.zero_tol * s0;
  int my_kmin = T, my_kz = 0;
  {
    double run = chunk[tid];
    for (int i = ce - 1; i >= cb; --i) {
      run = fma(sv[i], sv[i], run);
      if (run <= thr) my_kmin = i;
      if (sv[i] > zthr) ++my_kz;
    }
  }
  atomicMin(&kmin, my_kmin);
  atomicAdd(&kzero, my_kz);
  __syncthreads();
  int K = min(kmin, kzero);
  if (g.chi_max > 0) K = min(K, g.chi_max);
  K = min(K, g.keep_cap);
  K = min(K, T);
  K = max(K, 1);
  // tail weight at K
  if (K < T && K >= cb && K < ce) {
    double run = chunk[tid];
    for (int i = ce - 1; i >= K; --i) run = fma(sv[i], sv[i], run);
    disc_sh = run;
  }
  __syncthreads();
  if (K >= T && tid == 0) disc_sh = 0.0;
  for (int i = tid; i < K; i += nt) atomicAdd(&cnt[sk[i] >> 20], 1);
  __syncthreads();
  for (int s = tid; s < nsec; s += nt) kept[g.sec_begin + s] = cnt[s];
  if (tid == 0) {
    CutOut o;
    o.kept = K;
    o.flags = bad ? 1 : 0;
    o.discarded = disc_sh;
    o.total = W;
    o.margin = K < T ? (sv[K - 1] - sv[K]) / s0 : INFINITY;
    cut[gi] = o;
  }
}

// ---------------------------------------------------------------------------
// Update of B[s+1] and lambda[s+1]: one workgroup per new row.
__global__ void __launch_bounds__(256)
update_rows_kernel(const RowWork* __restrict__ rows, const SectorWork* __restrict__ secs,
                   const UpdateWork* __restrict__ upd, const double2* __restrict__ vh,
                   const double* __restrict__ sigma, const int* __restrict__ order) {
  const RowWork rw = rows[blockIdx.x];
  const SectorWork s = secs[rw.sector];
  const UpdateWork u = upd[rw.gate];
  const int src = order[s.sig + rw.j];
  const double2* xr = vh + s.off + (size_t)src * s.c;
  double2* dst = u.br_new + (size_t)rw.row * u.ldr;
  for (int col = threadIdx.x; col < u.ldr; col += blockDim.x) {
    const int cc = col - s.clo;
    dst[col] = (cc >= 0 && cc < s.c) ? xr[cc] : make_double2(0.0, 0.0);
  }
  if (threadIdx.x == 0) u.lam_new[rw.row] = sigma[s.sig + rw.j];
}

// Fill a list of device ranges with zeros (grid-stride per range).
__global__ void __launch_bounds__(256)
zero_fill_kernel(double2* const* __restrict__ ptrs, const long long* __restrict__ counts, int nranges) {
  for (int r = 0; r < nranges; ++r) {
    double2* p = ptrs[r];
    const long long n = counts[r];
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
      p[i] = make_double2(0.0, 0.0);
  }
}

// ---------------------------------------------------------------------------
// Generic batched complex GEMM, 32 x 32 tiles, k-chunks of 16 through LDS.
__global__ void __launch_bounds__(256)
zgemm_kernel(const GemmWork* __restrict__ probs, int nprob) {
  __shared__ double2 as[kGemmTile][17];
  __shared__ double2 bs[16][kGemmTile + 1];
  // locate the problem of this tile
  int lo = 0, hi = nprob - 1;
  const int tile = blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (probs[mid].tile_begin <= tile) lo = mid; else hi = mid - 1;
  }
  const GemmWork w = probs[lo];
  const int local = tile - w.tile_begin;
  const int tm = local / w.tiles_n, tn = local % w.tiles_n;
  const int row0 = tm * kGemmTile, col0 = tn * kGemmTile;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double2 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = make_double2(0.0, 0.0);
  for (int k0 = 0; k0 < w.k; k0 += 16) {
    for (int e = threadIdx.x; e < kGemmTile * 16; e += 256) {
      const int r = e >> 4, kk = e & 15;
      const int i = row0 + r, k = k0 + kk;
      double2 v = make_double2(0.0, 0.0);
      if (i < w.m && k < w.k)
        v = w.opa ? cconj(w.a[(size_t)k * w.lda + i]) : w.a[(size_t)i * w.lda + k];
      as[r][kk] = v;
    }
    for (int e = threadIdx.x; e < 16 * kGemmTile; e += 256) {
      const int kk = e >> 5, c = e & 31;
      const int j = col0 + c, k = k0 + kk;
      double2 v = make_double2(0.0, 0.0);
      if (j < w.n && k < w.k)
        v = w.opb ? cconj(w.b[(size_t)j * w.ldb + k]) : w.b[(size_t)k * w.ldb + j];
      bs[kk][c] = v;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < 16; ++kk) {
      const double2 a0 = as[ty][kk], a1 = as[ty + 16][kk];
      const double2 b0 = bs[kk][tx], b1 = bs[kk][tx + 16];
      cfma(acc[0][0], a0, b0);
      cfma(acc[0][1], a0, b1);
      cfma(acc[1][0], a1, b0);
      cfma(acc[1][1], a1, b1);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const int i = row0 + ty + 16 * a;
    if (i >= w.m) continue;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int j = col0 + tx + 16 * b;
      if (j >= w.n) continue;
      double2* cp = w.c + (size_t)i * w.ldc + j;
      double2 v = acc[a][b];
      if (w.beta_one) {
        const double2 o = *cp;
        v.x += o.x;
        v.y += o.y;
      }
      *cp = v;
    }
  }
}

// ---------------------------------------------------------------------------
// Amplitudes: one workgroup per pattern.  The charge path c_{s+1} = c_s - occ_s
// selects one block of every site tensor (Eq. (E2)); the amplitude is the
// product of those blocks.  Any missing charge gives exactly zero.
__global__ void __launch_bounds__(256)
amplitude_kernel(const double2* const* __restrict__ sites, const int* __restrict__ ld,
                 const int2* __restrict__ bondmap, const int* __restrict__ occ,
                 double2* __restrict__ out, int L, int d, int N, int maxdim) {
  extern __shared__ double2 vsm[];
  double2* v0 = vsm;
  double2* v1 = vsm + maxdim;
  __shared__ int ok;
  const int pat = blockIdx.x;
  const int* o = occ + (size_t)pat * L;
  if (threadIdx.x == 0) {
    int c = N, good = 1;
    for (int s = 0; s < L; ++s) {
      const int x = o[s];
      if (x < 0 || x >= d) { good = 0; break; }
      c -= x;
      if (c < 0) { good = 0; break; }
      if (bondmap[(size_t)(s + 1) * (N + 1) + c].y == 0) { good = 0; break; }
    }
    if (c != 0) good = 0;
    ok = good;
  }
  if (threadIdx.x == 0) v0[0] = make_double2(1.0, 0.0);
  __syncthreads();
  if (!ok) {
    if (threadIdx.x == 0) out[pat] = make_double2(0.0, 0.0);
    return;
  }
  int c = N;
  int n0 = 1, off0 = bondmap[c].x;   // bond 0 holds only charge N
  for (int s = 0; s < L; ++s) {
    const int c1 = c - o[s];
    const int2 b1 = bondmap[(size_t)(s + 1) * (N + 1) + c1];
    const double2* B = sites[s];
    const int lds = ld[s];
    for (int j = threadIdx.x; j < b1.y; j += blockDim.x) {
      double2 acc = make_double2(0.0, 0.0);
      for (int i = 0; i < n0; ++i) cfma(acc, v0[i], B[(size_t)(off0 + i) * lds + b1.x + j]);
      v1[j] = acc;
    }
    __syncthreads();
    double2* tmp = v0; v0 = v1; v1 = tmp;
    n0 = b1.y;
    off0 = b1.x;
    c = c1;
  }
  if (threadIdx.x == 0) out[pat] = v0[0];
}

// Gather kernels for re-truncation: dst[r][j] = src[r][map[j]] / src[map[r]][j].
__global__ void __launch_bounds__(256)
gather_cols_kernel(const double2* __restrict__ src, int lds, double2* __restrict__ dst, int ldd,
                   int rows, const int* __restrict__ map, int ncols) {
  const long long total = (long long)rows * ncols;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(e / ncols), j = (int)(e % ncols);
    dst[(size_t)r * ldd + j] = src[(size_t)r * lds + map[j]];
  }
}

__global__ void __launch_bounds__(256)
gather_rows_kernel(const double2* __restrict__ src, int lds, double2* __restrict__ dst, int ldd,
                   const int* __restrict__ map, int nrows, int cols) {
  const long long total = (long long)nrows * cols;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(e / cols), j = (int)(e % cols);
    dst[(size_t)r * ldd + j] = src[(size_t)map[r] * lds + j];
  }
}

__global__ void __launch_bounds__(256)
gather_vec_kernel(const double* __restrict__ src, double* __restrict__ dst,
                  const int* __restrict__ map, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[map[i]];
}

// ---------------------------------------------------------------------------
// Host launchers.

// ---------------------------------------------------------------------------
// Precision form of Theta formation: the charge-triple products on the matrix
// cores in split BF16, then the gate mix into the FP64 Theta workspaces.

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// x = hi + lo with hi = bf16(x), lo = bf16(x - hi): |x - hi - lo| <= 2^-18 |x|
// (after the float conversion of x, which adds 2^-24 |x|); BF16 bit patterns.
__device__ __forceinline__ void split_bf16(double x, unsigned short& hi, unsigned short& lo) {
  const float xf = (float)x;
  const __bf16 h = (__bf16)xf;
  const __bf16 l = (__bf16)(xf - (float)h);
  hi = __builtin_bit_cast(unsigned short, h);
  lo = __builtin_bit_cast(unsigned short, l);
}

__device__ __forceinline__ void split_store(unsigned short* out, long long plane, long long idx, double2 v) {
  unsigned short h, l;
  split_bf16(v.x, h, l);
  out[idx] = h;
  out[plane + idx] = l;
  split_bf16(v.y, h, l);
  out[2 * plane + idx] = h;
  out[3 * plane + idx] = l;
}

// The split pass: one 32 x 32 tile (rows x padded k) of one plan's planes per
// workgroup.  Rows are read along the frame's contiguous axis: directly for
// A planes, through an LDS transpose for the B planes.
__global__ void __launch_bounds__(256)
split_planes_kernel(const SplitPlanes* __restrict__ plans, int nplan, const int* __restrict__ ktab,
                    unsigned short* __restrict__ planes) {
  __shared__ double2 tile[kSpTile][kSpTile + 1];
  int lo = 0, hi = nplan - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (plans[mid].tile_begin <= (int)blockIdx.x) lo = mid; else hi = mid - 1;
  }
  const SplitPlanes w = plans[lo];
  const int local = blockIdx.x - w.tile_begin;
  const int r0 = (local / w.tiles_k) * kSpTile, kk0 = (local % w.tiles_k) * kSpTile;
  const int* kinv = ktab + w.kinv;
  unsigned short* out = planes + w.out;
  const long long plane = (long long)w.rows * w.ldk;
  const int t = threadIdx.x;
  if (!w.trans) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = r0 + (t >> 5) + 8 * q, kk = kk0 + (t & 31);
      if (i < w.rows && kk < w.ldk) {
        const int k = kinv[kk];
        const double2 v = k >= 0 ? w.src[(size_t)i * w.ld + k] : make_double2(0.0, 0.0);
        split_store(out, plane, (long long)i * w.ldk + kk, v);
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int kl = (t >> 5) + 8 * q, jl = t & 31;
      const int kk = kk0 + kl, j = r0 + jl;
      double2 v = make_double2(0.0, 0.0);
      if (kk < w.ldk && j < w.rows) {
        const int k = kinv[kk];
        if (k >= 0) v = w.src[(size_t)k * w.ld + j];
      }
      tile[kl][jl] = v;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int jl = (t >> 5) + 8 * q, kl = t & 31;
      const int j = r0 + jl, kk = kk0 + kl;
      if (j < w.rows && kk < w.ldk) split_store(out, plane, (long long)j * w.ldk + kk, tile[kl][jl]);
    }
  }
}

// LDS rows of one k chunk: 32 BF16 plus 8 of padding (80 bytes), so every
// 8-element operand read is one aligned 16-byte access.
constexpr int kSgRow = kSgK + 8;

// 16-byte groups (8 k) of a 64-row x 32-k chunk of one operand's 4 planes:
// 1024 groups, 4 per thread (group g = t + 256 q: plane g / 256, row
// (g % 256) / 4, k 8 (g % 4)); rows past `rows` and groups starting past `k`
// read as 0 (the planes are zero between charge blocks, so a group that
// starts inside the range is exact).
__device__ __forceinline__ void sg_fetch(uint4 (&r)[4], const unsigned short* __restrict__ base, long long pstride,
                                         int ld, int rows, int k, int row0, int k0) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int g = threadIdx.x + 256 * q;
    const int plane = g >> 8, row = (g & 255) >> 2, kg = 8 * (g & 3);
    r[q] = make_uint4(0u, 0u, 0u, 0u);
    if (row0 + row < rows && k0 + kg < k)
      r[q] = *reinterpret_cast<const uint4*>(base + plane * pstride + (size_t)(row0 + row) * ld + k0 + kg);
  }
}

__device__ __forceinline__ void sg_stage(const uint4 (&r)[4], unsigned short (*buf)[kSgTile][kSgRow]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int g = threadIdx.x + 256 * q;
    *reinterpret_cast<uint4*>(&buf[g >> 8][(g & 255) >> 2][8 * (g & 3)]) = r[q];
  }
}

__device__ __forceinline__ bf16x8 sg_op(const unsigned short (*buf)[kSgTile][kSgRow], int plane, int row, int k) {
  return *reinterpret_cast<const bf16x8*>(&buf[plane][row][k]);
}

// One 64 x 64 output tile per workgroup; wave w computes the 32 x 32 quadrant
// (rows 32 (w / 2), columns 32 (w % 2)) with v_mfma_f32_32x32x16_bf16.  Lane l
// supplies A[i = l % 32][k = 8 (l / 32) + e] and B[k = 8 (l / 32) + e][j = l % 32]
// (e = 0..7); its accumulator register r holds D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32].
// Per k step: Re = Ar Br - Ai Bi and Im = Ar Bi + Ai Br, each real product as
// hi*hi + hi*lo + lo*hi (the lo*lo term is below the split's error).  The k
// chunks go through two LDS buffers: the next chunk's loads are in flight
// during the products and are staged into the other buffer, one barrier per
// chunk.
__global__ void __launch_bounds__(256)
split_gemm_kernel(const SplitGemm* __restrict__ probs, int nprob) {
  __shared__ __align__(16) unsigned short sa[2][4][kSgTile][kSgRow];
  __shared__ __align__(16) unsigned short sb[2][4][kSgTile][kSgRow];
  int lo = 0, hi = nprob - 1;
  const int tile = blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (probs[mid].tile_begin <= tile) lo = mid; else hi = mid - 1;
  }
  const SplitGemm w = probs[lo];
  const int local = tile - w.tile_begin;
  const int row0 = (local / w.tiles_n) * kSgTile, col0 = (local % w.tiles_n) * kSgTile;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int R = 32 * (wave >> 1), Cq = 32 * (wave & 1);
  const int li = lane & 31, lk = 8 * (lane >> 5);
  f32x16 crp = {}, crn = {}, cim = {};
  uint4 ra[4], rb[4];
  sg_fetch(ra, w.a, w.pa, w.lda, w.m, w.k, row0, 0);
  sg_fetch(rb, w.b, w.pb, w.ldb, w.n, w.k, col0, 0);
  sg_stage(ra, sa[0]);
  sg_stage(rb, sb[0]);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < w.k; k0 += kSgK) {
    const bool more = k0 + kSgK < w.k;
    if (more) {
      sg_fetch(ra, w.a, w.pa, w.lda, w.m, w.k, row0, k0 + kSgK);
      sg_fetch(rb, w.b, w.pb, w.ldb, w.n, w.k, col0, k0 + kSgK);
    }
#pragma unroll
    for (int ks = 0; ks < kSgK; ks += 16) {
      const bf16x8 arh = sg_op(sa[buf], 0, R + li, ks + lk), arl = sg_op(sa[buf], 1, R + li, ks + lk);
      const bf16x8 aih = sg_op(sa[buf], 2, R + li, ks + lk), ail = sg_op(sa[buf], 3, R + li, ks + lk);
      const bf16x8 brh = sg_op(sb[buf], 0, Cq + li, ks + lk), brl = sg_op(sb[buf], 1, Cq + li, ks + lk);
      const bf16x8 bih = sg_op(sb[buf], 2, Cq + li, ks + lk), bil = sg_op(sb[buf], 3, Cq + li, ks + lk);
      crp = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arh, brh, crp, 0, 0, 0);
      crn = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aih, bih, crn, 0, 0, 0);
      cim = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arh, bih, cim, 0, 0, 0);
      crp = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arh, brl, crp, 0, 0, 0);
      crn = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aih, bil, crn, 0, 0, 0);
      cim = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arh, bil, cim, 0, 0, 0);
      crp = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arl, brh, crp, 0, 0, 0);
      crn = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ail, bih, crn, 0, 0, 0);
      cim = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arl, bih, cim, 0, 0, 0);
      cim = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aih, brh, cim, 0, 0, 0);
      cim = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aih, brl, cim, 0, 0, 0);
      cim = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ail, brh, cim, 0, 0, 0);
    }
    if (more) {
      // the other buffer was last read before the previous barrier
      sg_stage(ra, sa[buf ^ 1]);
      sg_stage(rb, sb[buf ^ 1]);
    }
    __syncthreads();
    buf ^= 1;
  }
  const int j = col0 + Cq + li;
  if (j < w.n) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = row0 + R + 8 * (r >> 2) + (lane >> 5) * 4 + (r & 3);
      if (i < w.m) w.c[(size_t)i * w.ldc + j] = make_float2(crp[r] - crn[r], cim[r]);
    }
  }
}

// Gate mix of the precision form: for the 32 x 32 tile of one charge pair,
// Theta~(cL, m, cR) = sum_j G^(n)[cL - m][a_j] P_j with the products P_j from
// the scratch (complex64, upcast), written like the plain kernel's epilogue.
__global__ void __launch_bounds__(256)
theta_mix_kernel(const GateWork* __restrict__ gates, const ThetaTile* __restrict__ tiles,
                 const SectorWork* __restrict__ secs, const double2* __restrict__ coef,
                 const float2* __restrict__ pbuf, double2* __restrict__ th_raw,
                 double2* __restrict__ th_scaled) {
  const ThetaTile& t = tiles[blockIdx.x];
  const GateWork g = gates[t.gate];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int nin = t.nin, nout = t.nout;
  for (int a = 0; a < 2; ++a) {
    const int r = ty + 16 * a;
    if (r >= t.nrow) continue;
    const double lam = g.lam_l[t.row0 + r];
    for (int b = 0; b < 2; ++b) {
      const int c = tx + 16 * b;
      if (c >= t.ncol) continue;
      double2 pv[kMaxD];
#pragma unroll
      for (int j = 0; j < kMaxD; ++j) {
        pv[j] = make_double2(0.0, 0.0);
        if (j < nin) {
          const float2 f = pbuf[t.poff[j] + (size_t)(t.pr0 + r) * t.ldp + t.pc0 + c];
          pv[j] = make_double2(f.x, f.y);
        }
      }
      for (int i = 0; i < nout; ++i) {
        double2 v = make_double2(0.0, 0.0);
#pragma unroll
        for (int j = 0; j < kMaxD; ++j)
          if (j < nin) cfma(v, coef[g.coef + (t.n * g.d + t.p[i]) * g.d + t.a[j]], pv[j]);
        const SectorWork s = secs[t.sec[i]];
        const size_t rr = (size_t)(t.orow[i] + r), cc = (size_t)(t.ocol[i] + c);
        th_raw[(size_t)s.off + rr * s.c + cc] = v;
        const size_t si = s.tall ? (size_t)s.off + cc * s.r + rr : (size_t)s.off + rr * s.c + cc;
        th_scaled[si] = make_double2(lam * v.x, lam * v.y);
      }
    }
  }
}

hipError_t launch_theta(const GateWork* gates, const ThetaTile* tiles, int ntiles,
                        const SectorWork* secs, const double2* coef, double2* raw,
                        double2* scaled, int maxw, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  if (maxw <= 4)
    hipLaunchKernelGGL(theta_kernel<4>, dim3(ntiles), dim3(256), 0, st, gates, tiles, secs, coef, raw, scaled);
  else
    hipLaunchKernelGGL(theta_kernel<kMaxD>, dim3(ntiles), dim3(256), 0, st, gates, tiles, secs, coef, raw, scaled);
  return hipGetLastError();
}

hipError_t launch_jacobi_init(const SectorWork* secs, const int* list, int count,
                              const double2* theta, double2* acc, JacobiOut* st, int* perm,
                              double* norm2, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(jacobi_init, dim3(count), dim3(256), 0, s, secs, list, theta, acc, st, perm, norm2);
  return hipGetLastError();
}

hipError_t launch_jacobi_sort(const SectorWork* secs, const int* list, int count, const JacobiOut* st,
                              int* perm, const double* norm2, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(jacobi_sort, dim3(count), dim3(256), 0, s, secs, list, st, perm, norm2);
  return hipGetLastError();
}

hipError_t launch_jacobi_step(const SectorWork* secs, const JacobiBlockWork* jb, int njb, int npairs,
                              int step, double2* theta, double2* acc, JacobiOut* st, const int* perm,
                              double* norm2, double tol, int max_inner, hipStream_t s) {
  if (npairs <= 0) return hipSuccess;
  hipLaunchKernelGGL(jacobi_block_step, dim3(npairs), dim3(256), 0, s, secs, jb, njb, step, theta, acc,
                     st, perm, norm2, tol, max_inner);
  return hipGetLastError();
}

hipError_t launch_jacobi_sweep_end(const int* list, int count, JacobiOut* st, int* active, hipStream_t s) {
  hipLaunchKernelGGL(jacobi_sweep_end, dim3(1), dim3(1024), 0, s, list, count, st, active);
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
  hipLaunchKernelGGL(jacobi_finalize, dim3(count), dim3(256), smem, s, secs, list, theta, acc, sigma, order);
  return hipGetLastError();
}

hipError_t launch_select(const GateWork* gates, int ngates, const SectorWork* secs,
                         const double* sigma, double* gsv, int* gsk, const long long* scratch_off,
                         int* kept, CutOut* cut, int maxP, hipStream_t st) {
  if (ngates <= 0) return hipSuccess;
  // LDS holds P doubles + P ints when P <= 4096 (48 KiB); larger goes to global scratch
  const int lds_cap = 4096;
  const int P = maxP <= lds_cap ? maxP : 0;
  const size_t smem = (size_t)P * (sizeof(double) + sizeof(int));
  hipLaunchKernelGGL(select_kernel, dim3(ngates), dim3(1024), smem, st, gates, secs, sigma, gsv,
                     gsk, scratch_off, kept, cut, P > 0 ? lds_cap : 0);
  return hipGetLastError();
}

hipError_t launch_update_rows(const RowWork* rows, int nrows, const SectorWork* secs,
                              const UpdateWork* upd, const double2* vh, const double* sigma,
                              const int* order, hipStream_t st) {
  if (nrows <= 0) return hipSuccess;
  hipLaunchKernelGGL(update_rows_kernel, dim3(nrows), dim3(256), 0, st, rows, secs, upd, vh, sigma, order);
  return hipGetLastError();
}

hipError_t launch_zero_fill(double2* const* ptrs, const long long* counts, int nranges,
                            long long maxcount, hipStream_t st) {
  if (nranges <= 0 || maxcount <= 0) return hipSuccess;
  long long blocks = (maxcount + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(zero_fill_kernel, dim3((unsigned)blocks), dim3(256), 0, st, ptrs, counts, nranges);
  return hipGetLastError();
}

hipError_t launch_zgemm(const GemmWork* probs, int nprob, int ntiles, hipStream_t st) {
  if (nprob <= 0 || ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(zgemm_kernel, dim3(ntiles), dim3(256), 0, st, probs, nprob);
  return hipGetLastError();
}

hipError_t launch_split_planes(const SplitPlanes* plans, int nplan, int ntiles, const int* ktab,
                               unsigned short* planes, hipStream_t st) {
  if (nplan <= 0 || ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(split_planes_kernel, dim3(ntiles), dim3(256), 0, st, plans, nplan, ktab, planes);
  return hipGetLastError();
}

hipError_t launch_split_gemm(const SplitGemm* probs, int nprob, int ntiles, hipStream_t st) {
  if (nprob <= 0 || ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(split_gemm_kernel, dim3(ntiles), dim3(256), 0, st, probs, nprob);
  return hipGetLastError();
}

hipError_t launch_theta_mix(const GateWork* gates, const ThetaTile* tiles, int ntiles, const SectorWork* secs,
                            const double2* coef, const float2* pbuf, double2* raw, double2* scaled, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(theta_mix_kernel, dim3(ntiles), dim3(256), 0, st, gates, tiles, secs, coef, pbuf, raw, scaled);
  return hipGetLastError();
}

hipError_t launch_amplitude(const double2* const* sites, const int* ld, const int2* bondmap,
                            const int* occ, double2* out, int count, int L, int d, int N,
                            int maxdim, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const size_t smem = (size_t)2 * maxdim * sizeof(double2);
  hipLaunchKernelGGL(amplitude_kernel, dim3(count), dim3(256), smem, st, sites, ld, bondmap, occ, out, L, d, N, maxdim);
  return hipGetLastError();
}

hipError_t launch_gather_cols(const double2* src, int lds, double2* dst, int ldd, int rows,
                              const int* map, int ncols, hipStream_t st) {
  const long long total = (long long)rows * ncols;
  if (total <= 0) return hipSuccess;
  long long blocks = (total + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(gather_cols_kernel, dim3((unsigned)blocks), dim3(256), 0, st, src, lds, dst, ldd, rows, map, ncols);
  return hipGetLastError();
}

hipError_t launch_gather_rows(const double2* src, int lds, double2* dst, int ldd, const int* map,
                              int nrows, int cols, hipStream_t st) {
  const long long total = (long long)nrows * cols;
  if (total <= 0) return hipSuccess;
  long long blocks = (total + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, st, src, lds, dst, ldd, map, nrows, cols);
  return hipGetLastError();
}

hipError_t launch_gather_vec(const double* src, double* dst, const int* map, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_vec_kernel, dim3((n + 255) / 256), dim3(256), 0, st, src, dst, map, n);
  return hipGetLastError();
}

}  // namespace u1mps
