// Launch wrappers of the gfx950 kernels (kernels.hip).  Every pointer is a
// device pointer; every launch goes to the given stream.
#pragma once

#include <mutex>

#include "internal.h"

namespace u1mps {

// tile_before[t] receives |lambda_s theta~|^2 of tile t before the gate.
hipError_t launch_theta(const GateWork* gates, const ThetaTile* tiles, int ntiles,
                        const SectorWork* secs, const double2* coef, double2* raw,
                        double2* scaled, double* tile_before, int maxw, hipStream_t st);

// Blocked one-sided Jacobi SVD of every listed sector (vectors: min(r, c)
// rows or columns of length max(r, c)); st holds per-sector state.
// perm and norm2 hold, per sector from its sigma offset, the vector order by
// descending norm and the vectors' squared norms.
hipError_t launch_jacobi_init(const SectorWork* secs, const int* list, int count,
                              const double2* theta, double2* acc, JacobiOut* st, int* perm,
                              double* norm2, hipStream_t s);
// One step launch over every block pair: step t of every sector's sweep
// (desync 0), or every sector's own step t mod (nb - 1) of its sweep
// t div (nb - 1) with the sweep ends folded in (desync 1; blocked: the sweep
// limit; ctr[0] counts the sectors still sweeping, ctr[1] those stopped
// unconverged; norm2 holds two buffers of nstride doubles, one per sweep
// parity).  Desynchronised launches need every sector's vector count at most
// jacobi_desync_rows(block).
int jacobi_desync_rows(int block);
hipError_t launch_jacobi_step(const SectorWork* secs, const JacobiPairWork* pairs, int npairs, int t,
                              int desync, int blocked, int* ctr, double2* theta, double2* acc, JacobiOut* st,
                              int* perm, double* norm2, long long nstride, double tol, int max_inner, int block,
                              hipStream_t s);
hipError_t launch_jacobi_sort(const SectorWork* secs, const int* list, int count, int maxrows, const JacobiOut* st,
                              int* perm, const double* norm2, hipStream_t s);
// active[0]: a sector still rotates; active[1]: the largest block count nbs[i]
// among those sectors (list order).
hipError_t launch_jacobi_sweep_end(const int* list, const int* nbs, int count, JacobiOut* st, int* active,
                                   hipStream_t s);
// Scalar sweeps on the vectors for sectors the blocked sweeps left unconverged.
hipError_t launch_jacobi_polish(const SectorWork* secs, const int* list, int count, double2* theta,
                                double2* acc, JacobiOut* st, double tol, int max_sweeps, hipStream_t s);
hipError_t launch_jacobi_finalize(const SectorWork* secs, const int* list, int count, int maxrows,
                                  double2* theta, const double2* acc, double* sigma, int* order,
                                  hipStream_t s);

// The cut's sort runs in LDS when every gate has at most kSelectLds candidate
// values, else (or when global is set) in the device scratch gsv/gsk.
// tile_before (may be NULL): per-tile weights before the gate, summed per gate
// into CutOut::leak.
hipError_t launch_select(const GateWork* gates, int ngates, const SectorWork* secs,
                         const double* sigma, double* gsv, int* gsk, const long long* scratch_off,
                         int* kept, CutOut* cut, int maxP, bool global, const double* tile_before,
                         hipStream_t st);

hipError_t launch_update_rows(const RowWork* rows, int nrows, const SectorWork* secs,
                              const UpdateWork* upd, const double2* vh, const double* sigma,
                              const int* order, hipStream_t st);

hipError_t launch_zero_fill(double2* const* ptrs, const long long* counts, int nranges,
                            long long maxcount, hipStream_t st);

// total (optional): a device count of the tiles to run, for lists planned on
// the device (ntiles is then an upper bound).
hipError_t launch_zgemm(const GemmWork* probs, int nprob, int ntiles, hipStream_t st, const int* total = nullptr);
// Precision form: split-BF16 charge-triple products into the complex64
// scratch, then the gate mix into the Theta workspaces.
hipError_t launch_split_planes(const SplitPlanes* plans, int nplan, int ntiles, const int* ktab,
                               unsigned short* planes, hipStream_t st);
// variant: the output tile shape, 0..kSgVariants-1 (kSgTileR x kSgTileC)
hipError_t launch_split_gemm(const SplitGemm* probs, int nprob, int ntiles, int variant, hipStream_t st);
hipError_t launch_theta_mix(const GateWork* gates, const ThetaTile* tiles, int ntiles, const SectorWork* secs,
                            const double2* coef, const double2* pbuf, double2* raw, double2* scaled,
                            double* tile_before, hipStream_t st);

// mod: 0 for a U(1) charge, n for a Z_n charge (bondmap then has n entries per bond).
hipError_t launch_amplitude(const double2* const* sites, const int* ld, const int2* bondmap,
                            const int* occ, double2* out, int count, int L, int d, int N, int mod,
                            int maxdim, Steps steps, hipStream_t st);

// Chain-rule sampling of `count` patterns (sample.hip): sites[s] (ldb[s]) and
// the left environments envs[s] (lde[s]) of every site, bondmap[(b, c)] =
// (offset, count) of charge c on bond b, uniforms[count * L]; writes occ and
// prob (-1 where a marginal vanished or was not finite).
// The sampler's round for one mode (sample.hip): gather of every group's
// vectors from the per-sample slots (column j of the maxblk x ld_slot slot
// matrix), then, after the two products, the draw of every sample.
// One round's plan on the device (one workgroup; nq <= kMaxSampleCharges):
// groups, product lists (nq * kMaxD entries each) and counts from the
// samples' charge positions on bond s+1.
hipError_t launch_sample_plan(const SampleCand* cand, int nq, const int* pos, int cnt, const double2* site, int ldb,
                              const double2* env, int lde, double2* vbuf, double2* wbuf, double2* xbuf, int* ids,
                              SampleGroup* groups, GemmWork* g1, GemmWork* g2, SampleCounts* counts, hipStream_t st);
hipError_t launch_sample_gather(const SampleGroup* groups, int ngroups, long long maxelems, const int* ids,
                                const double2* slots, int ld_slot, double2* vbuf, hipStream_t st);
// ntiles: an upper bound of sum over groups of ceil(ng / 16); the true count
// is counts->ptiles.  Writes every sample's new charge position into pos.
hipError_t launch_sample_pick(const SampleGroup* groups, int ngroups, int ntiles, const int* ids,
                              const double2* wbuf, const double2* xbuf, const double* uni, int L, int s,
                              double2* slots, int ld_slot, int* occ, double* prob, int* pos, SampleCounts* counts,
                              hipStream_t st);

hipError_t launch_gather_cols(const double2* src, int lds, double2* dst, int ldd, int rows,
                              const int* map, int ncols, hipStream_t st);
hipError_t launch_gather_rows(const double2* src, int lds, double2* dst, int ldd, const int* map,
                              int nrows, int cols, hipStream_t st);
hipError_t launch_gather_vec(const double* src, double* dst, const int* map, int n, hipStream_t st);

// Fixed device scratch of the entry point that allocates nothing
// (noalloc.hip): kScratchBytes per GPU.  scratch_region returns the array's
// device address on `device` (looked up once per device, with that device
// current); the caller holds scratch_lock() while it looks the address up
// and while its device work on the array runs.
constexpr size_t kScratchBytes = size_t(64) << 20;
std::unique_lock<std::mutex> scratch_lock();
hipError_t scratch_region(int device, void** ptr, size_t* bytes);

}  // namespace u1mps
