// Internal work-list records shared by the host runtime and the gfx950 kernels.
//
// Storage (all device, complex128 as double2):
//   site tensor B[s] = Gamma[s] * lambda[s+1] is a dense chi_s x chi_{s+1}
//   row-major "frame" whose rows (bond s) and columns (bond s+1) are sorted by
//   ascending right-charge.  Entries whose charge difference lies outside
//   0..d-1 are structural zeros (Eq. (E2)); kernels address only the allowed
//   blocks, and the update kernels write the zeros explicitly.  Because the
//   charges are sorted, every charge window [c, c+d-1] of a bond is one
//   contiguous index range, so each Theta(m) sector and each update block is
//   a strided submatrix.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace u1mps {

constexpr int kMaxD = 8;          // local dimension limit (occupations 0..7)
constexpr int kThetaTile = 32;    // Theta output tile edge
constexpr int kGemmTile = 32;     // generic ZGEMM tile edge
constexpr int kSelectLds = 4096;  // cut: candidate values sorted in LDS (48 KiB)

// One two-site update inside a batch.
struct GateWork {
  const double2* bl;      // B[s]   frame, chi_s x chi_{s+1}, row stride ldl
  const double2* br;      // B[s+1] frame, chi_{s+1} x chi_{s+2}, row stride ldr
  const double* lam_l;    // lambda of bond s (chi_s)
  int ldl, ldr;
  int coef;               // offset of this gate's (2d-1) x d x d coefficients
  int d;
  int sec_begin, sec_end; // sector range [begin, end) in the batch's sector list
  int tile_begin, tile_end;  // Theta tile range [begin, end) of this gate
  int keep_cap;           // largest admissible new bond dimension
  int chi_max;            // <= 0: none
  double cutoff;
  double zero_tol;
};

// The charge of every local state (an entry of a site tensor on local state p
// joins a left charge cL to the right charge cL - s[p]); U(1) and Z_n: s[p] = p.
struct Steps {
  int s[kMaxD];
};

// One middle-charge sector Theta(m) of one gate.
struct SectorWork {
  int gate;               // index into the batch's GateWork list
  int m;                  // middle charge
  int r, c;               // Theta(m) is r x c
  int rlo, clo;           // first row (bond s index) / column (bond s+2 index) of the first block
  long long off;          // element offset of Theta(m) in the theta workspaces
  int sig;                // offset of this sector's r singular values / row order
  int kmax;               // min(r, c): at most this many values enter the cut
  int tall;               // r > c: the SVD orthogonalises the c columns instead
  long long acc;          // tall only: element offset of the c x c rotation accumulator
  // the rows of Theta(m) are row blocks of the bond-s frame and its columns
  // column blocks of the bond-(s+2) frame, packed in ascending charge order:
  // block k covers frame rows rb_off[k] .. rb_off[k] + rb_n[k] - 1 at rows
  // rb_pos[k] .. of Theta(m) (likewise cb_* for columns).  U(1) and Z_n
  // sectors are one block each way; two U(1) components give several.
  int nrb, ncb;
  int rb_off[kMaxD], rb_n[kMaxD], rb_pos[kMaxD];
  int cb_off[kMaxD], cb_n[kMaxD], cb_pos[kMaxD];
};

// One 32x32 output tile of one (cL, cR) charge pair of one gate.  The tile
// accumulates the products B[s](cL, cM) B[s+1](cM, cR) for every middle
// charge cM of the old bond that lies in the window, then mixes them with
// the gate block G^(n), n = cL - cR, into every new sector m of the window.
struct ThetaTile {
  int gate;
  int row0, nrow;         // rows of the tile, bond s index space
  int col0, ncol;         // columns of the tile, bond s+2 index space
  int n;                  // total local photon number of the pair
  int nin, nout;
  int k0[kMaxD], kn[kMaxD], a[kMaxD];      // input segments: start, length, cL - cM
  int sec[kMaxD], p[kMaxD];                // output sector, cL - m
  int orow[kMaxD], ocol[kMaxD];            // tile origin inside Theta(m)
  // split-BF16 form only: the products P_j = B[s](cL, segment j) B[s+1](., cR)
  // of the tile's charge pair sit in the complex128 scratch at poff[j], row-major
  // with row length ldp (= the pair's column count); the tile starts at
  // row pr0, column pc0 of them
  long long poff[kMaxD];
  int pr0, pc0, ldp;
};

// Split-BF16 form.  Before the products, each gate's two site tensors are
// split into kSgPlanes BF16 planes (re hi, re mid, re lo, im hi, im mid,
// im lo; x = hi + mid + lo with hi = bf16(x), mid = bf16(x - hi),
// lo = bf16(x - hi - mid)) over a padded k axis (the middle bond,
// every charge block starting at a multiple of 8, zeros between blocks):
// A planes hold B[s] (rows = bond s), B planes hold B[s+1] transposed
// (rows = bond s+2), so both operands have k contiguous.
constexpr int kSgVariants = 4;    // output tiles of the products: 64x64, 32x64, 64x32, 32x32
constexpr int kSgTileR[kSgVariants] = {64, 32, 64, 32};
constexpr int kSgTileC[kSgVariants] = {64, 64, 32, 32};
constexpr int kSgK = 32;          // k chunk staged per step
constexpr int kSpTile = 32;       // tile edge of the split pass
constexpr int kSgPlanes = 6;      // BF16 planes per operand: 3 parts x (re, im)

struct SplitPlanes {
  const double2* src;     // the site frame
  int ld;                 // its row stride
  int rows;               // output rows (A: chi_s; B: chi_{s+2})
  int trans;              // 0: out[i][kk] = src[i][k]; 1: out[j][kk] = src[k][j]
  int ldk;                // padded k extent, a multiple of 8
  long long kinv;         // offset in the batch's k table: source k of each padded kk, -1 = pad
  long long out;          // offset (elements) of plane 0; plane p at out + p * rows * ldk
  int tiles_k;            // ceil(ldk / kSpTile)
  int tile_begin;
};

// One charge-triple product C (m x n, complex128, row-major, ldc) = A (m x k) B
// (k x n) from the planes: a and b point at plane 0 of the operands' first
// row and first k (k contiguous, row strides lda and ldb, multiples of 8),
// plane strides pa and pb.
struct SplitGemm {
  const unsigned short* a;
  const unsigned short* b;
  double2* c;
  long long pa, pb;
  int m, n, k;
  int lda, ldb, ldc;
  int tiles_n[kSgVariants];     // per tile shape: ceil(n / tile columns)
  int tile_begin[kSgVariants];  // per tile shape: first flattened tile of this problem
};

// A generic complex GEMM problem C = op(A) op(B) (+ C when beta_one).
// op 0 = as stored (row-major), op 1 = conjugate transpose of the stored matrix.
struct GemmWork {
  const double2* a;
  const double2* b;
  double2* c;
  int m, n, k;
  int lda, ldb, ldc;
  int opa, opb;
  int beta_one;
  int tiles_n;            // ceil(n / kGemmTile)
  int tile_begin;         // first flattened tile of this problem
};

// One group of the sampler's round for mode s: the samples standing on one
// charge c of bond s+1 (ids[id0 .. id0 + ng - 1]), their vectors gathered
// into V (nc x ng, row-major) at voff; for each candidate local state loc[k]
// with a block of charge c + step on bond s (nr[k] rows), W_k = B_s[.] V and
// X_k = E_s[.] W_k (nr[k] x ng, row-major) at woff[k] of their buffers.
struct SampleGroup {
  int nc, ng, id0, nout;
  int tile0;              // first workgroup of the group in the draw kernel (16 samples each)
  long long voff;
  int loc[kMaxD], nr[kMaxD];
  int pos[kMaxD];         // charge position on bond s of candidate k's block
  long long woff[kMaxD];
};

// The fixed part of a group, per charge position q of bond s+1 (the sampler
// plans each round on the device from these and the samples' positions):
// the block of q (nc rows, frame offset off1 on bond s+1) and, for every
// local state with a block on bond s, that block's position, rows and frame
// offset on bond s.
struct SampleCand {
  int nc, off1, nout;
  int loc[kMaxD], pos[kMaxD], nr[kMaxD], off0[kMaxD];
};

// Charge positions per bond the sampler's device plan handles (LDS counters).
constexpr int kMaxSampleCharges = 1024;

// Per-round totals the device plan writes for the launches that follow
// (whose grids are host-side upper bounds), and a sticky failure flag.
struct SampleCounts {
  int nt1, nt2, ptiles, failed;
};

// New-row descriptor for the update of B[s+1] and lambda[s+1].
struct RowWork {
  int gate;               // GateWork index (for the output pointers)
  int sector;             // SectorWork index
  int j;                  // rank inside the sector (0 = largest value)
  int row;                // row of the new frame
};

// Output pointers of one gate's update.
struct UpdateWork {
  double2* br_new;        // new B[s+1] frame, chi' x chi_{s+2}, stride ldr
  double* lam_new;        // new lambda (chi')
  int ldr;                // chi_{s+2}
};

// Result of the cut of one gate, written by the select kernel.
struct CutOut {
  int kept;
  int flags;              // bit 0: vanished/non-finite
  double discarded;
  double total;
  double margin;
  double leak;            // weight the local cutoff removed: |lambda theta~|^2 before
                          // the gate minus the total weight after it
};

// Blocked Jacobi: vectors are grouped in blocks of kJB8 = 8 or kJB = 16
// (mps_opts.jacobi_block); one round-robin step pairs the nb blocks of a
// sector into nb/2 block pairs, each handled by one workgroup.
constexpr int kJB = 16;
constexpr int kJP = 2 * kJB;
constexpr int kJB8 = 8;

// One block pair of a round-robin step: workgroup p of a step launch takes
// entry p (the pairs of all sectors, heaviest sector first).
struct JacobiPairWork {
  int sector;             // SectorWork index
  int nb;                 // the sector's number of blocks, even (an empty block pads odd counts)
  int k;                  // pair index within the sector's step (0 .. nb/2 - 1)
  int pad;
};

// Per-sector Jacobi state and statistics.
struct JacobiOut {
  int sweeps;             // sweeps in which the sector was still active
  int rotations;          // block pairs rotated, summed over sweeps
  int converged;
  int rot3[3];            // block pairs rotated in sweep w, at rot3[w % 3] (lockstep launches: rot3[0])
  unsigned long long gram_units;    // sum over evaluated pairs of nv^2 * len
  unsigned long long apply_units;   // sum over rotated pairs of nv^2 * (len + tall accumulator len)
  double fro2;            // squared Frobenius norm of the sector (rotation invariant)
};

}  // namespace u1mps
