// Exact sampling of output patterns of the U(1) MPS (gfx950).
//
// A pattern i_1..i_L is drawn with probability |c_i|^2 / <psi|psi>, c_i the
// amplitude of Eq. (E2), by the chain rule from the last mode to the first:
// with v the contraction B_{s+1} .. B_{L-1} of the occupations already drawn
// (a vector on one charge block of bond s+1), occupation i of mode s has the
// unnormalised conditional probability
//     p_i = w_i^dagger E_s w_i,   w_i = B_s[charge c + step_i, charge c] v,
// E_s the left environment of bond s (block-diagonal by charge, built by the
// norm's contraction), step_i the charge of local state i (U(1): i).  The
// occupation is the smallest i whose cumulative p exceeds u * sum(p) for the
// caller's uniform u; v becomes w_i / sqrt(p_i).  With a Z_n charge (mod = n)
// the charges add mod n.
//
// All samples advance together, one mode per round.  The samples that stand
// on the same charge c of bond s+1 form a group: their vectors are gathered
// into the columns of one matrix V (sample_gather_kernel), so that W_i =
// B_s[c + step_i, c] V and X_i = E_s[c + step_i] W_i are two products with
// many right-hand sides (the generic complex GEMM) and every block of B_s and
// E_s is read once per group instead of once per sample; sample_pick_kernel
// then forms p_i = Re(W_i^dagger X_i) column by column, draws, and writes the
// sample's new vector into its slot and its new charge position.  The rounds
// are planned on the device (sample_plan_kernel: the groups and the product
// lists from the samples' charge positions), so the host enqueues all of them
// without waiting; the product and draw launches take host-side upper bounds
// on their grids and the true totals from the plan.
#include "device_util.h"
#include "kernels.h"

namespace u1mps {

constexpr int kPickS = 16;
constexpr int kPickRows = 256 / kPickS;

// Plan of one round (one workgroup): the samples' charge positions on bond
// s+1 are counted per position in LDS; thread 0 lays out the groups in
// position order (offsets of V, W and X, the draw kernel's tiles, the first
// tile of every group in the two product lists); then thread q writes group
// q, thread q * kMaxD + k the product entries of candidate k of group q,
// W_k = B_s[block k, block q] V and X_k = E_s[block k] W_k (entries without a
// candidate hold no tiles, so the lists keep a fixed length of nq * kMaxD),
// and every sample takes a slot in its group.  The order of the samples inside
// a group is arbitrary: every sample's column of the products, its draw and
// its new vector depend on its own column only.
__global__ void __launch_bounds__(1024)
sample_plan_kernel(const SampleCand* __restrict__ cand, int nq, const int* __restrict__ pos, int cnt,
                   const double2* __restrict__ site, int ldb, const double2* __restrict__ env, int lde,
                   double2* vbuf, double2* wbuf, double2* xbuf, int* __restrict__ ids,
                   SampleGroup* __restrict__ groups, GemmWork* __restrict__ g1, GemmWork* __restrict__ g2,
                   SampleCounts* __restrict__ counts) {
  __shared__ int hist[kMaxSampleCharges];
  __shared__ int id0s[kMaxSampleCharges], tile0s[kMaxSampleCharges], gt0[kMaxSampleCharges];
  __shared__ long long voffs[kMaxSampleCharges], woffs[kMaxSampleCharges];
  for (int q = threadIdx.x; q < nq; q += blockDim.x) hist[q] = 0;
  __syncthreads();
  for (int j = threadIdx.x; j < cnt; j += blockDim.x) atomicAdd(&hist[pos[j]], 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    int id0 = 0, tile0 = 0, t = 0;
    long long voff = 0, woff = 0;
    for (int q = 0; q < nq; ++q) {
      const SampleCand& c = cand[q];
      const int ng = hist[q], tn = (ng + kGemmTile - 1) / kGemmTile;
      id0s[q] = id0;
      tile0s[q] = tile0;
      gt0[q] = t;
      voffs[q] = voff;
      woffs[q] = woff;
      for (int k = 0; k < c.nout; ++k) {
        t += ((c.nr[k] + kGemmTile - 1) / kGemmTile) * tn;
        woff += (long long)c.nr[k] * ng;
      }
      voff += (long long)c.nc * ng;
      id0 += ng;
      tile0 += (ng + kPickS - 1) / kPickS;
    }
    counts->nt1 = t;
    counts->nt2 = t;                         // the two lists have the same shapes
    counts->ptiles = tile0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nq * kMaxD; e += blockDim.x) {
    const int q = e / kMaxD, k = e % kMaxD;
    const SampleCand& c = cand[q];
    const int ng = hist[q], tn = (ng + kGemmTile - 1) / kGemmTile;
    // this entry's first tile and W offset: the group's plus its earlier candidates'
    int tb = gt0[q];
    long long wo = woffs[q];
    for (int k2 = 0; k2 < k && k2 < c.nout; ++k2) {
      tb += ((c.nr[k2] + kGemmTile - 1) / kGemmTile) * tn;
      wo += (long long)c.nr[k2] * ng;
    }
    GemmWork a, b;
    a.opa = a.opb = b.opa = b.opb = 0;
    a.beta_one = b.beta_one = 0;
    a.a = b.a = nullptr;
    a.b = b.b = nullptr;
    a.c = b.c = nullptr;
    a.m = a.n = a.k = b.m = b.n = b.k = 0;
    a.lda = a.ldb = a.ldc = b.lda = b.ldb = b.ldc = 0;
    a.tiles_n = b.tiles_n = 0;
    a.tile_begin = b.tile_begin = tb;
    if (k < c.nout) {
      const int nr = c.nr[k];
      a.a = site + (size_t)c.off0[k] * ldb + c.off1;
      a.lda = ldb;
      a.b = vbuf + voffs[q];
      a.ldb = ng;
      a.c = wbuf + wo;
      a.ldc = ng;
      a.m = nr;
      a.n = ng;
      a.k = c.nc;
      a.tiles_n = tn;
      b.a = env + (size_t)c.off0[k] * lde + c.off0[k];
      b.lda = lde;
      b.b = wbuf + wo;
      b.ldb = ng;
      b.c = xbuf + wo;
      b.ldc = ng;
      b.m = nr;
      b.n = ng;
      b.k = nr;
      b.tiles_n = tn;
    }
    g1[e] = a;
    g2[e] = b;
  }
  for (int q = threadIdx.x; q < nq; q += blockDim.x) {
    const SampleCand& c = cand[q];
    const int ng = hist[q];
    SampleGroup g;
    g.nc = c.nc;
    g.ng = ng;
    g.id0 = id0s[q];
    g.nout = c.nout;
    g.tile0 = tile0s[q];
    g.voff = voffs[q];
    long long wo = woffs[q];
    for (int k = 0; k < kMaxD; ++k) {
      const bool on = k < c.nout;
      g.loc[k] = on ? c.loc[k] : 0;
      g.nr[k] = on ? c.nr[k] : 0;
      g.pos[k] = on ? c.pos[k] : 0;
      g.woff[k] = on ? wo : 0;
      if (on) wo += (long long)c.nr[k] * ng;
    }
    groups[q] = g;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < cnt; j += blockDim.x) ids[atomicAdd(&id0s[pos[j]], 1)] = j;
}

// V_g[k][jj] = slots[k][ids[id0 + jj]] for every group (blockIdx.y), k < nc.
__global__ void __launch_bounds__(256)
sample_gather_kernel(const SampleGroup* __restrict__ groups, const int* __restrict__ ids,
                     const double2* __restrict__ slots, int ld_slot, double2* __restrict__ vbuf) {
  const SampleGroup g = groups[blockIdx.y];
  const long long n = (long long)g.nc * g.ng;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(e / g.ng), jj = (int)(e % g.ng);
    vbuf[g.voff + e] = slots[(size_t)k * ld_slot + ids[g.id0 + jj]];
  }
}

// One workgroup per kPickS consecutive samples of one group (columns jj0 ..
// jj0 + kPickS - 1): thread t takes sample column jj0 + t % kPickS and every
// kPickRows-th row starting at t / kPickS, so each row's kPickS columns are
// one contiguous load.  The candidate probabilities p_k = Re sum_r
// conj(W_k[r][jj]) X_k[r][jj] are summed over the row slices in LDS (fixed
// order); the first slice draws (NaN or a non-positive total leaves pick -1)
// and updates the running probability; every slice then writes its rows of
// the new vector W_pick[:, jj] / sqrt(p_pick) into the sample's slot.
__global__ void __launch_bounds__(256)
sample_pick_kernel(const SampleGroup* __restrict__ groups, int ngroups, const int* __restrict__ ids,
                   const double2* __restrict__ wbuf, const double2* __restrict__ xbuf,
                   const double* __restrict__ uni, int L, int s, double2* __restrict__ slots, int ld_slot,
                   int* __restrict__ occ, double* __restrict__ prob, int* __restrict__ pos,
                   SampleCounts* __restrict__ counts) {
  __shared__ double part[kPickRows][kMaxD][kPickS];
  __shared__ int pick_sh[kPickS];
  __shared__ double scale_sh[kPickS];
  const int b = blockIdx.x;
  if (b >= counts->ptiles) return;          // the grid is an upper bound
  int lo = 0, hi = ngroups - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (groups[mid].tile0 <= b) lo = mid; else hi = mid - 1;
  }
  const SampleGroup& g = groups[lo];
  const int col = threadIdx.x % kPickS, slice = threadIdx.x / kPickS;
  const int jj = (b - g.tile0) * kPickS + col;
  const bool live = jj < g.ng;
  const int nout = g.nout, ng = g.ng;
  for (int k = 0; k < nout; ++k) {
    double q = 0.0;
    if (live) {
      const double2* w = wbuf + g.woff[k] + jj;
      const double2* x = xbuf + g.woff[k] + jj;
      for (int r = slice; r < g.nr[k]; r += kPickRows) {
        const double2 a = w[(size_t)r * ng], c = x[(size_t)r * ng];
        q = fma(a.x, c.x, fma(a.y, c.y, q));
      }
    }
    part[slice][k][col] = q;
  }
  __syncthreads();
  if (slice == 0) {
    int pick = -1;
    double sc = 0.0;
    if (live) {
      const int j = ids[g.id0 + jj];
      double pv[kMaxD];
      double tot = 0.0;
      for (int k = 0; k < nout; ++k) {
        double q = 0.0;
        for (int r = 0; r < kPickRows; ++r) q += part[r][k][col];
        pv[k] = (q > 0.0 || q != q) ? q : 0.0;     // rounding below zero -> 0; NaN kept
        tot += pv[k];
      }
      if (tot > 0.0 && tot <= DBL_MAX) {
        const double ut = uni[(size_t)j * L + s] * tot;
        double acc = 0.0;
        for (int k = 0; k < nout; ++k) {
          acc += pv[k];
          if (ut < acc) {
            pick = k;
            break;
          }
        }
        if (pick < 0)
          for (int k = nout - 1; k >= 0; --k)
            if (pv[k] > 0.0) {
              pick = k;
              break;
            }
      }
      if (pick >= 0) {
        prob[j] *= pv[pick] / tot;
        occ[(size_t)j * L + s] = g.loc[pick];
        sc = 1.0 / sqrt(pv[pick]);
      }
      // a vanished or non-finite marginal fails the call; the sample keeps a
      // valid position so that the later rounds stay in bounds
      pos[j] = pick >= 0 ? g.pos[pick] : 0;
      if (pick < 0) atomicOr(&counts->failed, 1);
    }
    pick_sh[col] = pick;
    scale_sh[col] = sc;
  }
  __syncthreads();
  const int pick = pick_sh[col];
  if (!live || pick < 0) return;
  const int j = ids[g.id0 + jj];
  const double sc = scale_sh[col];
  const double2* w = wbuf + g.woff[pick] + jj;
  for (int r = slice; r < g.nr[pick]; r += kPickRows) {
    const double2 a = w[(size_t)r * ng];
    slots[(size_t)r * ld_slot + j] = make_double2(a.x * sc, a.y * sc);
  }
}

hipError_t launch_sample_plan(const SampleCand* cand, int nq, const int* pos, int cnt, const double2* site, int ldb,
                              const double2* env, int lde, double2* vbuf, double2* wbuf, double2* xbuf, int* ids,
                              SampleGroup* groups, GemmWork* g1, GemmWork* g2, SampleCounts* counts, hipStream_t st) {
  if (nq <= 0 || nq > kMaxSampleCharges) return hipErrorInvalidValue;
  hipLaunchKernelGGL(sample_plan_kernel, dim3(1), dim3(1024), 0, st, cand, nq, pos, cnt, site, ldb, env, lde, vbuf,
                     wbuf, xbuf, ids, groups, g1, g2, counts);
  return hipGetLastError();
}

hipError_t launch_sample_gather(const SampleGroup* groups, int ngroups, long long maxelems, const int* ids,
                                const double2* slots, int ld_slot, double2* vbuf, hipStream_t st) {
  if (ngroups <= 0 || maxelems <= 0) return hipSuccess;
  long long bx = (maxelems + 255) / 256;
  if (bx > 1024) bx = 1024;
  hipLaunchKernelGGL(sample_gather_kernel, dim3((unsigned)bx, (unsigned)ngroups), dim3(256), 0, st, groups, ids,
                     slots, ld_slot, vbuf);
  return hipGetLastError();
}

hipError_t launch_sample_pick(const SampleGroup* groups, int ngroups, int ntiles, const int* ids,
                              const double2* wbuf, const double2* xbuf, const double* uni, int L, int s,
                              double2* slots, int ld_slot, int* occ, double* prob, int* pos, SampleCounts* counts,
                              hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(sample_pick_kernel, dim3(ntiles), dim3(256), 0, st, groups, ngroups, ids, wbuf, xbuf, uni, L,
                     s, slots, ld_slot, occ, prob, pos, counts);
  return hipGetLastError();
}

}  // namespace u1mps
