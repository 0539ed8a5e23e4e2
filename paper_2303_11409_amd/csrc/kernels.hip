// Cut, update and read-out kernels of the U(1)-symmetric MPS engine
// (Sec. II, Eqs. (E1)-(E4)):
//   select_kernel  one cut over all sectors of a gate: sort, discarded-weight
//                  rule, chi cap, kept count per sector (FP64).
//   update_*       new B[s+1] = kept V^dagger rows, lambda = kept values,
//                  new B[s] = Theta~ V_kept (generic complex GEMM).
//   amplitude_kernel, gather_*  amplitudes of occupation patterns (Eq. (E1))
//                  and the gathers of truncation and norm contraction.
// Wave64 throughout: reductions use cross-lane shuffles over 64 lanes.
#include "device_util.h"
#include "kernels.h"

namespace u1mps {

// ---------------------------------------------------------------------------
// Cut over all sectors of one gate.  One workgroup of 512 threads per gate
// (LDS: the candidates, up to 48 KiB, plus 12 KiB of counters and sums).  Entries are
// (value, key) with key = local sector << 20 | rank; they are sorted by value
// descending, then key ascending (bitonic network), and the kept count is
//   K = max(1, min(K_eps, K_zero, chi_max, keep_cap, T)).
// The weights behind K_eps and the discarded weight are compensated sums.
__device__ __forceinline__ bool sel_before(double va, int ka, double vb, int kb) {
  return va > vb || (va == vb && ka < kb);
}

// Compensated FP64 sums (double-double accumulation): a value is hi + lo.
// add_sq adds v^2 exactly up to the final rounding: the product's rounding
// error comes from an fma, the sum's from TwoSum, both folded into lo.
struct Dd {
  double hi, lo;
};
__device__ __forceinline__ Dd dd_add(Dd a, double b) {
  const double s = a.hi + b;
  const double bb = s - a.hi;
  const double err = (a.hi - (s - bb)) + (b - bb);
  return {s, a.lo + err};
}
__device__ __forceinline__ Dd dd_add_sq(Dd a, double v) {
  const double p = v * v;
  const double pe = fma(v, v, -p);
  Dd r = dd_add(a, p);
  r.lo += pe;
  return r;
}
__device__ __forceinline__ Dd dd_add(Dd a, Dd b) {
  Dd r = dd_add(a, b.hi);
  r.lo += b.lo;
  return r;
}
__device__ __forceinline__ double dd_val(Dd a) { return a.hi + a.lo; }

constexpr int kSelectThreads = 512;

__global__ void __launch_bounds__(kSelectThreads)
select_kernel(const GateWork* __restrict__ gates, const SectorWork* __restrict__ secs,
              const double* __restrict__ sigma, double* __restrict__ gsv, int* __restrict__ gsk,
              const long long* __restrict__ scratch_off, int* __restrict__ kept,
              CutOut* __restrict__ cut, int lds_cap, const double* __restrict__ tile_before) {
  extern __shared__ double ssm[];
  __shared__ int cnt[1024];
  __shared__ Dd chunk[kSelectThreads];
  __shared__ int kmin, kzero, nf_flag;
  __shared__ Dd disc_sh;
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
  // chunked compensated sums of squares over the T valid entries, in sorted order
  const int C = (T + nt - 1) / nt;
  const int cb = tid * C, ce = min(T, cb + C);
  Dd part = {0.0, 0.0};
  int nonfinite = 0;
  for (int i = cb; i < ce; ++i) {
    const double v = sv[i];
    if (!isfinite(v)) nonfinite = 1;
    part = dd_add_sq(part, v);
  }
  chunk[tid] = part;
  if (tid == 0) { kmin = T; kzero = 0; nf_flag = 0; }
  __syncthreads();
  if (nonfinite) atomicOr(&nf_flag, 1);
  __syncthreads();
  if (nf_flag) bad = true;
  if (tid == 0) {
    // suffix sums of the chunk sums, fixed order
    Dd run = {0.0, 0.0};
    for (int t = nt - 1; t >= 0; --t) {
      const Dd v = chunk[t];
      chunk[t] = run;          // sum of chunks after t
      run = dd_add(run, v);
    }
    disc_sh = run;             // temporarily: total weight W
  }
  __syncthreads();
  const double W = dd_val(disc_sh);
  const double thr = g.cutoff * W;
  const double zthr = g.zero_tol * s0;
  int my_kmin = T, my_kz = 0;
  {
    Dd run = chunk[tid];
    for (int i = ce - 1; i >= cb; --i) {
      run = dd_add_sq(run, sv[i]);
      if (dd_val(run) <= thr) my_kmin = i;
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
    Dd run = chunk[tid];
    for (int i = ce - 1; i >= K; --i) run = dd_add_sq(run, sv[i]);
    disc_sh = run;
  }
  __syncthreads();
  if (K >= T && tid == 0) disc_sh = Dd{0.0, 0.0};
  for (int i = tid; i < K; i += nt) atomicAdd(&cnt[sk[i] >> 20], 1);
  // weight before the gate: the gate's tile sums in a fixed order
  Dd bsum = {0.0, 0.0};
  if (tile_before) {
    const int nts = g.tile_end - g.tile_begin;
    const int TC = (nts + nt - 1) / nt;
    for (int i = g.tile_begin + tid * TC; i < min(g.tile_end, g.tile_begin + (tid + 1) * TC); ++i)
      bsum = dd_add(bsum, tile_before[i]);
  }
  __syncthreads();
  chunk[tid] = bsum;
  __syncthreads();
  if (tid == 0) {
    Dd b = {0.0, 0.0};
    for (int t = 0; t < nt; ++t) b = dd_add(b, chunk[t]);
    chunk[0] = b;
  }
  __syncthreads();
  for (int s = tid; s < nsec; s += nt) kept[g.sec_begin + s] = cnt[s];
  if (tid == 0) {
    CutOut o;
    o.kept = K;
    o.flags = bad ? 1 : 0;
    o.discarded = dd_val(disc_sh);
    o.total = W;
    o.margin = K < T ? (sv[K - 1] - sv[K]) / s0 : INFINITY;
    o.leak = tile_before ? dd_val(chunk[0]) - W : 0.0;
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
  const SectorWork& s = secs[rw.sector];
  const UpdateWork u = upd[rw.gate];
  const int src = order[s.sig + rw.j];
  const double2* xr = vh + s.off + (size_t)src * s.c;
  double2* dst = u.br_new + (size_t)rw.row * u.ldr;
  // the sector's columns are its column blocks of the frame; zero elsewhere
  const int ncb = s.ncb;
  for (int col = threadIdx.x; col < u.ldr; col += blockDim.x) dst[col] = make_double2(0.0, 0.0);
  // the zeros land before the blocks overwrite their columns (workgroup-scope fence)
  __syncthreads();
  for (int k = 0; k < ncb; ++k) {
    const int off = s.cb_off[k], n = s.cb_n[k], pos = s.cb_pos[k];
    for (int c = threadIdx.x; c < n; c += blockDim.x) dst[off + c] = xr[pos + c];
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
zgemm_kernel(const GemmWork* __restrict__ probs, int nprob, const int* __restrict__ total) {
  __shared__ double2 as[kGemmTile][17];
  __shared__ double2 bs[16][kGemmTile + 1];
  const int tile = blockIdx.x;
  // a list planned on the device: the grid is an upper bound, *total the tiles
  if (total && tile >= *total) return;
  // locate the problem of this tile (problems without tiles are never found:
  // the last problem whose first tile is <= tile has it)
  int lo = 0, hi = nprob - 1;
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
// Amplitudes: one workgroup per pattern.  The charge path c_{s+1} = c_s -
// step[occ_s] (mod n for a Z_n charge) selects one block of every site tensor
// (Eq. (E2)); the amplitude is the product of those blocks.  Any missing
// charge gives exactly zero.  bondmap has nc = (mod ? mod : N + 1) entries per
// bond (N: the charge of bond 0, the largest of all).
__global__ void __launch_bounds__(256)
amplitude_kernel(const double2* const* __restrict__ sites, const int* __restrict__ ld,
                 const int2* __restrict__ bondmap, const int* __restrict__ occ,
                 double2* __restrict__ out, int L, int d, int N, int mod, int maxdim, Steps st) {
  const int nc = mod ? mod : N + 1;
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
      c = mod ? (c - x + mod) % mod : c - st.s[x];
      if (c < 0 || c >= nc) { good = 0; break; }
      if (bondmap[(size_t)(s + 1) * nc + c].y == 0) { good = 0; break; }
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
    const int c1 = mod ? (c - o[s] + mod) % mod : c - st.s[o[s]];
    const int2 b1 = bondmap[(size_t)(s + 1) * nc + c1];
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

hipError_t launch_select(const GateWork* gates, int ngates, const SectorWork* secs,
                         const double* sigma, double* gsv, int* gsk, const long long* scratch_off,
                         int* kept, CutOut* cut, int maxP, bool global, const double* tile_before,
                         hipStream_t st) {
  if (ngates <= 0) return hipSuccess;
  // LDS holds P doubles + P ints when P <= kSelectLds (48 KiB); larger goes to global scratch
  const int P = (maxP <= kSelectLds && !global) ? maxP : 0;
  const size_t smem = (size_t)P * (sizeof(double) + sizeof(int));
  hipLaunchKernelGGL(select_kernel, dim3(ngates), dim3(kSelectThreads), smem, st, gates, secs, sigma, gsv,
                     gsk, scratch_off, kept, cut, P > 0 ? kSelectLds : 0, tile_before);
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

hipError_t launch_zgemm(const GemmWork* probs, int nprob, int ntiles, hipStream_t st, const int* total) {
  if (nprob <= 0 || ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(zgemm_kernel, dim3(ntiles), dim3(256), 0, st, probs, nprob, total);
  return hipGetLastError();
}

hipError_t launch_amplitude(const double2* const* sites, const int* ld, const int2* bondmap,
                            const int* occ, double2* out, int count, int L, int d, int N, int mod,
                            int maxdim, Steps steps, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const size_t smem = (size_t)2 * maxdim * sizeof(double2);
  hipLaunchKernelGGL(amplitude_kernel, dim3(count), dim3(256), smem, st, sites, ld, bondmap, occ, out, L, d, N, mod,
                     maxdim, steps);
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
