// Theta formation of the two-site update on sites (s, s+1) (Sec. II, the
// two-site tensor of Eq. (E2) under a photon-number-conserving gate):
//   theta_kernel        Theta~(cL, m, cR) = sum_cM G^(n)[(cL-m), (cL-cM)] B[s](cL,cM) B[s+1](cM,cR)
//                       (charge-sector-matched products in complex128, the gate
//                       mixed per n = cL - cR in the epilogue), plus
//                       Theta = lambda_s * Theta~, the input of the SVD.
//   split_planes_kernel, split_gemm_kernel, theta_mix_kernel
//                       the same in the split-BF16 form: BF16 planes of the
//                       site tensors, the charge-triple products on the matrix
//                       cores (FP32 accumulation), the gate mix in FP64.
#include "device_util.h"
#include "kernels.h"

namespace u1mps {

// ---------------------------------------------------------------------------
// Theta formation.  One workgroup (256 threads, 16 x 16) per 32 x 32 tile of
// one (cL, cR) pair; each thread owns rows ty, ty+16 and columns tx, tx+16.
// Sum over the workgroup's 256 threads in a fixed order (deterministic).
__device__ __forceinline__ double block_sum256(double v, double* red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

template <int W>
__global__ void __launch_bounds__(256)
theta_kernel(const GateWork* __restrict__ gates, const ThetaTile* __restrict__ tiles,
             const SectorWork* __restrict__ secs, const double2* __restrict__ coef,
             double2* __restrict__ th_raw, double2* __restrict__ th_scaled,
             double* __restrict__ tile_before) {
  __shared__ ThetaTile t;
  __shared__ double2 as[kThetaTile][17];
  __shared__ double2 bs[16][kThetaTile + 1];
  __shared__ double red[4];
  if (threadIdx.x == 0) t = tiles[blockIdx.x];
  __syncthreads();
  const GateWork g = gates[t.gate];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  // lambda_s of this thread's two rows (0 past the tile)
  double lr[2];
#pragma unroll
  for (int a = 0; a < 2; ++a) lr[a] = ty + 16 * a < t.nrow ? g.lam_l[t.row0 + ty + 16 * a] : 0.0;
  double before = 0.0;     // |lambda_s P_j|^2 summed over the input segments

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
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        before = fma(lr[a] * lr[a], fma(p[a][b].x, p[a][b].x, p[a][b].y * p[a][b].y), before);
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
  before = block_sum256(before, red);
  if (threadIdx.x == 0) tile_before[blockIdx.x] = before;
}


// ---------------------------------------------------------------------------
// Precision form of Theta formation: the charge-triple products on the matrix
// cores in split BF16, then the gate mix into the FP64 Theta workspaces.

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// x = hi + mid + lo in BF16 (8 significant bits each): hi = bf16(x),
// mid = bf16(x - hi), lo = bf16(x - hi - mid), the differences taken in FP64
// (exact: each part agrees with what remains to its leading bits) and each
// part rounded through FP32.  Every rounding keeps the next 8 bits of what
// remains, so |x - hi| <= 2^-8 |x|, |x - hi - mid| <= 2^-16 |x| and
// |x - hi - mid - lo| <= 2^-24 |x| (up to the FP32 step, 2^-24 of each part).
__device__ __forceinline__ void split_bf16(double x, unsigned short& hi, unsigned short& mid,
                                           unsigned short& lo) {
  const __bf16 h = (__bf16)(float)x;
  const double r1 = x - (double)(float)h;
  const __bf16 m = (__bf16)(float)r1;
  const double r2 = r1 - (double)(float)m;
  const __bf16 l = (__bf16)(float)r2;
  hi = __builtin_bit_cast(unsigned short, h);
  mid = __builtin_bit_cast(unsigned short, m);
  lo = __builtin_bit_cast(unsigned short, l);
}

// Four consecutive padded-k entries of one row into the six planes (re hi,
// re mid, re lo, im hi, im mid, im lo), one 8-byte store per plane (idx is a
// multiple of 4).
__device__ __forceinline__ void split_store4(unsigned short* out, long long plane, long long idx,
                                             const double2 (&v)[4]) {
  ushort4 p[kSgPlanes];
  split_bf16(v[0].x, p[0].x, p[1].x, p[2].x); split_bf16(v[0].y, p[3].x, p[4].x, p[5].x);
  split_bf16(v[1].x, p[0].y, p[1].y, p[2].y); split_bf16(v[1].y, p[3].y, p[4].y, p[5].y);
  split_bf16(v[2].x, p[0].z, p[1].z, p[2].z); split_bf16(v[2].y, p[3].z, p[4].z, p[5].z);
  split_bf16(v[3].x, p[0].w, p[1].w, p[2].w); split_bf16(v[3].y, p[3].w, p[4].w, p[5].w);
#pragma unroll
  for (int q = 0; q < kSgPlanes; ++q) *reinterpret_cast<ushort4*>(out + q * plane + idx) = p[q];
}

// The split pass: one 32 x 32 tile (rows x padded k) of one plan's planes per
// workgroup; thread t covers row t / 8 and the four padded k entries
// 4 (t % 8) .. 4 (t % 8) + 3 (ldk is a multiple of 8, so such a group is
// either inside the row or past its end).  Rows are read along the frame's
// contiguous axis: directly for A planes, through an LDS transpose for the B
// planes.
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
  const int row = r0 + (t >> 3), kl = 4 * (t & 7), kk = kk0 + kl;
  double2 v[4];
  if (!w.trans) {
    if (row < w.rows && kk < w.ldk) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int k = kinv[kk + e];
        v[e] = k >= 0 ? w.src[(size_t)row * w.ld + k] : make_double2(0.0, 0.0);
      }
      split_store4(out, plane, (long long)row * w.ldk + kk, v);
    }
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int tl = (t >> 5) + 8 * q, jl = t & 31;    // tile row = padded k, column = output row
      const int kq = kk0 + tl, j = r0 + jl;
      double2 x = make_double2(0.0, 0.0);
      if (kq < w.ldk && j < w.rows) {
        const int k = kinv[kq];
        if (k >= 0) x = w.src[(size_t)k * w.ld + j];
      }
      tile[tl][jl] = x;
    }
    __syncthreads();
    if (row < w.rows && kk < w.ldk) {
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] = tile[kl + e][t >> 3];
      split_store4(out, plane, (long long)row * w.ldk + kk, v);
    }
  }
}

// LDS rows of one k chunk: 32 BF16 plus 8 of padding (80 bytes), so every
// 8-element operand read is one aligned 16-byte access.  Two buffers of six
// planes per operand: 120 KiB of LDS per workgroup for a 64 x 64 tile.
constexpr int kSgRow = kSgK + 8;

// 16-byte groups (8 k) of a ROWS-row x 32-k chunk of one operand's six
// planes: 6 * 4 * ROWS groups over the NT threads of the workgroup (group g:
// plane g / (4 ROWS), row (g % (4 ROWS)) / 4, k 8 (g % 4)); rows past `rows`
// and groups starting past `k` read as 0 (the planes are zero between charge
// blocks, so a group that starts inside the range is exact).
template <int ROWS, int NT>
struct SgLoad {
  static constexpr int kGroups = kSgPlanes * 4 * ROWS;
  static constexpr int kPer = (kGroups + NT - 1) / NT;
  uint4 r[kPer];
  __device__ __forceinline__ void fetch(const unsigned short* __restrict__ base, long long pstride, int ld,
                                        int rows, int k, int row0, int k0) {
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int g = threadIdx.x + NT * q;
      const int plane = g / (4 * ROWS), row = (g % (4 * ROWS)) >> 2, kg = 8 * (g & 3);
      r[q] = make_uint4(0u, 0u, 0u, 0u);
      if (g < kGroups && row0 + row < rows && k0 + kg < k)
        r[q] = *reinterpret_cast<const uint4*>(base + plane * pstride + (size_t)(row0 + row) * ld + k0 + kg);
    }
  }
  __device__ __forceinline__ void stage(unsigned short (*buf)[ROWS][kSgRow]) const {
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int g = threadIdx.x + NT * q;
      if (g < kGroups)
        *reinterpret_cast<uint4*>(&buf[g / (4 * ROWS)][(g % (4 * ROWS)) >> 2][8 * (g & 3)]) = r[q];
    }
  }
};

template <int ROWS>
__device__ __forceinline__ bf16x8 sg_op(const unsigned short (*buf)[ROWS][kSgRow], int plane, int row, int k) {
  return *reinterpret_cast<const bf16x8*>(&buf[plane][row][k]);
}

// The split products of one real product x y, x = x[0] + x[1] + x[2] and
// y = y[0] + y[1] + y[2] (hi, mid, lo): the leading term x0 y0 into `big`,
// the seven terms x_i y_j with 0 < i + j <= 3 into `small` (only lo lo, below
// 2^-32 of |x||y|, is dropped).  Keeping the corrections apart from the
// leading term means the FP32 rounding of their sum is relative to the
// corrections, 2^-8 of the product, not to the product.
__device__ __forceinline__ void sg_real8(const bf16x8* x, const bf16x8* y, f32x16& big, f32x16& small) {
  big = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x[0], y[0], big, 0, 0, 0);
  small = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x[0], y[1], small, 0, 0, 0);
  small = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x[1], y[0], small, 0, 0, 0);
  small = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x[0], y[2], small, 0, 0, 0);
  small = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x[2], y[0], small, 0, 0, 0);
  small = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x[1], y[1], small, 0, 0, 0);
  small = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x[1], y[2], small, 0, 0, 0);
  small = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x[2], y[1], small, 0, 0, 0);
}

// The parts with their signs flipped (bit 15 of every BF16).
__device__ __forceinline__ void sg_negate3(const bf16x8* x, bf16x8* out) {
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    u32x4 v = __builtin_bit_cast(u32x4, x[p]);
    v ^= 0x80008000u;
    out[p] = __builtin_bit_cast(bf16x8, v);
  }
}

// One (32 WR) x (32 WC) output tile per workgroup of WR x WC waves; wave w
// computes the 32 x 32 quadrant (rows 32 (w / WC), columns 32 (w % WC)) with
// v_mfma_f32_32x32x16_bf16.  Lane l supplies A[i = l % 32][k = 8 (l / 32) + e]
// and B[k = 8 (l / 32) + e][j = l % 32] (e = 0..7); its accumulator register r
// holds D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32].  Per k step: Re = Ar Br +
// Ai (-Bi) and Im = Ar Bi + Ai Br, each real product as the split terms of
// sg_real8, into four accumulators (Re and Im, leading terms and corrections)
// whose chains interleave.  Products of BF16 values are exact in FP32; the
// matrix cores accumulate one 32-wide k chunk in FP32, the chunk sums are
// added in FP64 (so FP32 rounding grows with the chunk, not with k), and the
// product is stored in complex128.  Every output element sees the same sequence of
// matrix-core operations whatever the tile shape, so the shapes give bitwise
// the same products (the tuner picks one by speed alone).  The k chunks go
// through two LDS buffers: the next chunk's loads are in flight during the
// products and are staged into the other buffer, one barrier per chunk.
template <int WR, int WC>
__global__ void __launch_bounds__(64 * WR * WC)
split_gemm_kernel(const SplitGemm* __restrict__ probs, int nprob, int variant) {
  constexpr int NT = 64 * WR * WC, TR = 32 * WR, TC = 32 * WC;
  __shared__ __align__(16) unsigned short sa[2][kSgPlanes][TR][kSgRow];
  __shared__ __align__(16) unsigned short sb[2][kSgPlanes][TC][kSgRow];
  int lo = 0, hi = nprob - 1;
  const int tile = blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (probs[mid].tile_begin[variant] <= tile) lo = mid; else hi = mid - 1;
  }
  const SplitGemm w = probs[lo];
  const int tn = w.tiles_n[variant];
  const int local = tile - w.tile_begin[variant];
  const int row0 = (local / tn) * TR, col0 = (local % tn) * TC;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int R = 32 * (wave / WC), Cq = 32 * (wave % WC);
  const int li = lane & 31, lk = 8 * (lane >> 5);
  double dre[16], dim[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) dre[r] = dim[r] = 0.0;
  SgLoad<TR, NT> la;
  SgLoad<TC, NT> lb;
  la.fetch(w.a, w.pa, w.lda, w.m, w.k, row0, 0);
  lb.fetch(w.b, w.pb, w.ldb, w.n, w.k, col0, 0);
  la.stage(sa[0]);
  lb.stage(sb[0]);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < w.k; k0 += kSgK) {
    const bool more = k0 + kSgK < w.k;
    if (more) {
      la.fetch(w.a, w.pa, w.lda, w.m, w.k, row0, k0 + kSgK);
      lb.fetch(w.b, w.pb, w.ldb, w.n, w.k, col0, k0 + kSgK);
    }
    // the second k step of a chunk that ends the segment early is all zero
    const int nks = k0 + 16 < w.k ? 2 : 1;
    f32x16 reb = {}, res = {}, imb = {}, ims = {};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (h >= nks) break;
      // planes 0..2: re hi, mid, lo; 3..5: im hi, mid, lo
      bf16x8 a[kSgPlanes], b[kSgPlanes], bin[3];
#pragma unroll
      for (int p = 0; p < kSgPlanes; ++p) {
        a[p] = sg_op<TR>(sa[buf], p, R + li, 16 * h + lk);
        b[p] = sg_op<TC>(sb[buf], p, Cq + li, 16 * h + lk);
      }
      sg_negate3(b + 3, bin);
      sg_real8(a, b, reb, res);
      sg_real8(a + 3, bin, reb, res);
      sg_real8(a, b + 3, imb, ims);
      sg_real8(a + 3, b, imb, ims);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      dre[r] += (double)reb[r] + (double)res[r];
      dim[r] += (double)imb[r] + (double)ims[r];
    }
    if (more) {
      // the other buffer was last read before the previous barrier
      la.stage(sa[buf ^ 1]);
      lb.stage(sb[buf ^ 1]);
    }
    __syncthreads();
    buf ^= 1;
  }
  const int j = col0 + Cq + li;
  if (j < w.n) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = row0 + R + 8 * (r >> 2) + (lane >> 5) * 4 + (r & 3);
      if (i < w.m) w.c[(size_t)i * w.ldc + j] = make_double2(dre[r], dim[r]);
    }
  }
}

// Gate mix of the precision form: for the 32 x 32 tile of one charge pair,
// Theta~(cL, m, cR) = sum_j G^(n)[cL - m][a_j] P_j with the products P_j from
// the complex128 scratch, written like the plain kernel's epilogue.
__global__ void __launch_bounds__(256)
theta_mix_kernel(const GateWork* __restrict__ gates, const ThetaTile* __restrict__ tiles,
                 const SectorWork* __restrict__ secs, const double2* __restrict__ coef,
                 const double2* __restrict__ pbuf, double2* __restrict__ th_raw,
                 double2* __restrict__ th_scaled, double* __restrict__ tile_before) {
  __shared__ double red[4];
  const ThetaTile& t = tiles[blockIdx.x];
  const GateWork g = gates[t.gate];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int nin = t.nin, nout = t.nout;
  double before = 0.0;     // |lambda_s P_j|^2 summed over the input segments
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
          pv[j] = pbuf[t.poff[j] + (size_t)(t.pr0 + r) * t.ldp + t.pc0 + c];
          before = fma(lam * lam, fma(pv[j].x, pv[j].x, pv[j].y * pv[j].y), before);
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
  before = block_sum256(before, red);
  if (threadIdx.x == 0) tile_before[blockIdx.x] = before;
}


// ---------------------------------------------------------------------------
// Host launchers.

hipError_t launch_theta(const GateWork* gates, const ThetaTile* tiles, int ntiles,
                        const SectorWork* secs, const double2* coef, double2* raw,
                        double2* scaled, double* tile_before, int maxw, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  if (maxw <= 4)
    hipLaunchKernelGGL(theta_kernel<4>, dim3(ntiles), dim3(256), 0, st, gates, tiles, secs, coef, raw, scaled,
                       tile_before);
  else
    hipLaunchKernelGGL(theta_kernel<kMaxD>, dim3(ntiles), dim3(256), 0, st, gates, tiles, secs, coef, raw, scaled,
                       tile_before);
  return hipGetLastError();
}

hipError_t launch_split_planes(const SplitPlanes* plans, int nplan, int ntiles, const int* ktab,
                               unsigned short* planes, hipStream_t st) {
  if (nplan <= 0 || ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(split_planes_kernel, dim3(ntiles), dim3(256), 0, st, plans, nplan, ktab, planes);
  return hipGetLastError();
}

hipError_t launch_split_gemm(const SplitGemm* probs, int nprob, int ntiles, int variant, hipStream_t st) {
  if (nprob <= 0 || ntiles <= 0) return hipSuccess;
  switch (variant) {
    case 0:
      hipLaunchKernelGGL((split_gemm_kernel<2, 2>), dim3(ntiles), dim3(256), 0, st, probs, nprob, variant);
      break;
    case 1:
      hipLaunchKernelGGL((split_gemm_kernel<1, 2>), dim3(ntiles), dim3(128), 0, st, probs, nprob, variant);
      break;
    case 2:
      hipLaunchKernelGGL((split_gemm_kernel<2, 1>), dim3(ntiles), dim3(128), 0, st, probs, nprob, variant);
      break;
    case 3:
      hipLaunchKernelGGL((split_gemm_kernel<1, 1>), dim3(ntiles), dim3(64), 0, st, probs, nprob, variant);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_theta_mix(const GateWork* gates, const ThetaTile* tiles, int ntiles, const SectorWork* secs,
                            const double2* coef, const double2* pbuf, double2* raw, double2* scaled,
                            double* tile_before, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(theta_mix_kernel, dim3(ntiles), dim3(256), 0, st, gates, tiles, secs, coef, pbuf, raw, scaled,
                     tile_before);
  return hipGetLastError();
}

}  // namespace u1mps
