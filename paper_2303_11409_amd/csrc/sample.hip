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
// One workgroup (four waves) per sample.  Each matrix-vector product gives
// every row of the block to a group of g lanes, g the power of two covering
// the vector (at most 64), so short blocks keep the wave busy with several
// rows; the groups read their row contiguously.
#include "device_util.h"
#include "kernels.h"

namespace u1mps {

__device__ __forceinline__ int group_width(int n) {
  int g = 1;
  while (g < n && g < 64) g <<= 1;
  return g;
}

__device__ __forceinline__ double group_sum(double v, int g) {
  for (int o = g >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// y[r] = sum_k A[r * lda + k] x[k] for r < nr, k < nk (x and y in LDS).
__device__ void block_matvec(const double2* __restrict__ A, int lda, int nr, int nk,
                             const double2* x, double2* y) {
  const int g = group_width(nk);
  const int lane = threadIdx.x & 63;
  const int sub = lane & (g - 1);
  const int row0 = (threadIdx.x >> 6) * (64 / g) + lane / g;
  const int step = (blockDim.x >> 6) * (64 / g);
  for (int rb = 0; rb < nr; rb += step) {
    const int r = rb + row0;
    double2 acc = make_double2(0.0, 0.0);
    if (r < nr)
      for (int k = sub; k < nk; k += g) cfma(acc, A[(size_t)r * lda + k], x[k]);
    acc.x = group_sum(acc.x, g);
    acc.y = group_sum(acc.y, g);
    if (r < nr && sub == 0) y[r] = acc;
  }
}

// This thread's share of Re sum_r conj(x[r]) sum_k A[r * lda + k] x[k].
__device__ double block_quad(const double2* __restrict__ A, int lda, int n, const double2* x) {
  const int g = group_width(n);
  const int lane = threadIdx.x & 63;
  const int sub = lane & (g - 1);
  const int row0 = (threadIdx.x >> 6) * (64 / g) + lane / g;
  const int step = (blockDim.x >> 6) * (64 / g);
  double q = 0.0;
  for (int rb = 0; rb < n; rb += step) {
    const int r = rb + row0;
    double2 acc = make_double2(0.0, 0.0);
    if (r < n)
      for (int k = sub; k < n; k += g) cfma(acc, A[(size_t)r * lda + k], x[k]);
    acc.x = group_sum(acc.x, g);
    acc.y = group_sum(acc.y, g);
    if (r < n && sub == 0) q += x[r].x * acc.x + x[r].y * acc.y;
  }
  return q;
}

__global__ void __launch_bounds__(256)
sample_kernel(const double2* const* __restrict__ sites, const int* __restrict__ ldb,
              const double2* const* __restrict__ envs, const int* __restrict__ lde,
              const int2* __restrict__ bondmap, const double* __restrict__ uni, int* __restrict__ occ,
              double* __restrict__ prob, int L, int d, int N, int mod, int maxblk, Steps st) {
  const int ncb = mod ? mod : N + 1;             // bondmap entries per bond
  extern __shared__ double2 smem[];
  double2* v = smem;
  double2* w = smem + maxblk;
  __shared__ double part[4];
  __shared__ double pv[kMaxD];
  __shared__ int pick_sh;
  const int j = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (tid == 0) v[0] = make_double2(1.0, 0.0);
  int c = 0;                                   // charge of bond s+1; bond L holds only 0
  int nc = 1, offc = bondmap[(size_t)L * ncb].x;
  double pr = 1.0;
  __syncthreads();
  for (int s = L - 1; s >= 0; --s) {
    const double2* B = sites[s];
    const int lb = ldb[s];
    const double2* E = envs[s];
    const int le = lde[s];
    for (int i = 0; i < d; ++i) {
      const int c2 = mod ? (c + i) % mod : c + st.s[i];
      const int2 bm = c2 < ncb ? bondmap[(size_t)s * ncb + c2] : make_int2(0, 0);
      double q = 0.0;
      if (bm.y > 0) {
        block_matvec(B + (size_t)bm.x * lb + offc, lb, bm.y, nc, v, w);
        __syncthreads();
        q = block_quad(E + (size_t)bm.x * le + bm.x, le, bm.y, w);
      }
      q = wave_sum(q);
      if (lane == 0) part[wv] = q;
      __syncthreads();
      if (tid == 0) {
        const double t = part[0] + part[1] + part[2] + part[3];
        pv[i] = (t > 0.0 || t != t) ? t : 0.0;   // rounding below zero -> 0; NaN kept
      }
      __syncthreads();
    }
    if (tid == 0) {
      double tot = 0.0;
      for (int i = 0; i < d; ++i) tot += pv[i];
      int pick = -1;
      if (tot > 0.0 && tot <= DBL_MAX) {
        const double ut = uni[(size_t)j * L + s] * tot;
        double acc = 0.0;
        for (int i = 0; i < d; ++i) {
          acc += pv[i];
          if (ut < acc) {
            pick = i;
            break;
          }
        }
        if (pick < 0)
          for (int i = d - 1; i >= 0; --i)
            if (pv[i] > 0.0) {
              pick = i;
              break;
            }
        pr *= pv[pick] / tot;
      }
      pick_sh = pick;
    }
    __syncthreads();
    const int i = pick_sh;
    if (i < 0) {                                // the whole workgroup leaves together
      if (tid == 0) prob[j] = -1.0;
      return;
    }
    const int cn = mod ? (c + i) % mod : c + st.s[i];
    const int2 bm = bondmap[(size_t)s * ncb + cn];
    block_matvec(B + (size_t)bm.x * lb + offc, lb, bm.y, nc, v, w);
    __syncthreads();
    const double sc = 1.0 / sqrt(pv[i]);
    for (int r = tid; r < bm.y; r += blockDim.x) v[r] = make_double2(w[r].x * sc, w[r].y * sc);
    if (tid == 0) occ[(size_t)j * L + s] = i;
    c = cn;
    nc = bm.y;
    offc = bm.x;
    __syncthreads();
  }
  if (tid == 0) prob[j] = pr;
}

hipError_t launch_sample(const double2* const* sites, const int* ldb, const double2* const* envs,
                         const int* lde, const int2* bondmap, const double* uniforms, int* occ,
                         double* prob, int count, int L, int d, int N, int mod, int maxblk, Steps steps,
                         hipStream_t st) {
  if (count <= 0) return hipSuccess;
  if (d > kMaxD || (size_t)2 * maxblk * sizeof(double2) > kSampleLds) return hipErrorInvalidValue;
  hipLaunchKernelGGL(sample_kernel, dim3(count), dim3(256), 2 * maxblk * sizeof(double2), st, sites, ldb,
                     envs, lde, bondmap, uniforms, occ, prob, L, d, N, mod, maxblk, steps);
  return hipGetLastError();
}

}  // namespace u1mps
