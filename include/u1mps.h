/*
 * u1mps.h -- C ABI of the MI355X (gfx950) U(1)-symmetric MPS gate engine.
 *
 * The library applies photon-number-conserving two-mode gates (beam
 * splitters of a linear-optics circuit) to a matrix-product state whose bond
 * indices carry right-charge labels, and reads out amplitudes and norms.
 *
 * What is computed follows Sec. II of "Towards Symmetry-Aware Efficient
 * Simulation of Quantum Systems and Beyond" (arXiv 2303.11409).  (E1)-(E4)
 * name the four displayed relations of that section in order: the Vidal-form
 * amplitude, the U(1) amplitude with Kronecker deltas, the right-charge
 * definition, and the charge balance with its boundary values.
 *
 *   - the state is the Vidal-form MPS of Eq. (E1), sites 0..L-1 (the paper's
 *     1..M), bonds 0..L, bond b between site b-1 and site b;
 *   - every bond index alpha carries its right-charge c_b(alpha), the number
 *     of photons on sites b..L-1 (Eq. (E3)); the Kronecker deltas of Eq. (E2)
 *     fix the physical index of site s to c_s(alpha) - c_{s+1}(beta), so site
 *     tensors carry no physical index; boundary charges are c_0 = N and
 *     c_L = 0 (Eq. (E4));
 *   - a two-site update builds Theta(m) for every middle charge m, takes its
 *     SVD, and keeps the largest singular values over all m together, at most
 *     chi of them (the block-sparse SVDs of Sec. II).
 *
 * Conventions shared by every call
 * --------------------------------
 *   Complex numbers cross the boundary as mps_z (two doubles, re then im).
 *   Every array argument is a HOST pointer unless stated otherwise; the
 *   library copies inputs before it returns and never keeps caller memory.
 *   The caller owns every output array; the library owns mps_t and all
 *   device memory it obtained through mps_device.
 *   A mode unitary u2 is 2x2 row-major {u00, u01, u10, u11} and maps creation
 *   operators column-wise: a0^+ -> u00 a0^+ + u10 a1^+, a1^+ -> u01 a0^+ +
 *   u11 a1^+.  A gate on `site` acts on modes site and site+1.
 *   Errors: every call returns an mps_status; MPS_OK is 0, errors are
 *   negative.  Argument and charge errors are detected before any state
 *   changes.  A device-side failure of an update (Jacobi non-convergence, a
 *   vanished or non-finite two-site matrix) and an allocation failure are
 *   reported by the call that detects them, before the update writes the
 *   state: the state is unchanged.  After MPS_E_DEVICE (a failed HIP call) the
 *   state is unspecified and the handle should be destroyed.
 *   mps_last_error() returns a thread-local message for the last failure.
 *   One handle must not be used from two threads at once.
 */
#ifndef U1MPS_H
#define U1MPS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mps_state* mps_t;
typedef struct { double re, im; } mps_z;

typedef enum {
  MPS_OK = 0,
  MPS_E_ARG = -1,      /* bad argument (range, NULL, overlapping gates, ...)      */
  MPS_E_CHARGE = -2,   /* charge labels violate Eqs. (E2)-(E4)                     */
  MPS_E_NOMEM = -3,    /* the allocator returned NULL                              */
  MPS_E_DEVICE = -4,   /* a HIP runtime call failed                                */
  MPS_E_NOCONV = -5,   /* a Jacobi SVD did not converge within max_sweeps          */
  MPS_E_NUMERIC = -6   /* a two-site matrix vanished or held a non-finite value    */
} mps_status;

/* Device memory and stream hooks.  alloc(bytes, ctx) returns a device
 * pointer (NULL on failure); release(ptr, ctx) returns it.  Both may be NULL,
 * in which case hipMalloc/hipFree are used.  `stream` is a hipStream_t on
 * which every kernel and copy of the handle is issued (NULL: the null
 * stream).  The struct is copied by mps_create. */
typedef struct {
  void* (*alloc)(size_t bytes, void* ctx);
  void (*release)(void* ptr, void* ctx);
  void* ctx;
  void* stream;
} mps_device;

/* Truncation and solver options.
 *   chi_max    cap on every bond dimension (Sec. II's chi); <= 0 means none.
 *   cutoff     eps of the discarded-weight rule: keep the smallest K with
 *              sum_{i>=K} s_i^2 <= eps * sum_i s_i^2 over the singular values
 *              of all sectors of one two-site update; 0 disables it.
 *   zero_tol   singular values <= zero_tol * s_max are dropped as numerical
 *              zeros (default 1e-13).
 *   max_sweeps Jacobi sweep limit per sector (default 40): blocked sweeps
 *              first (at most blocked_sweeps, default 32), then scalar sweeps
 *              on the vectors of any sector still rotating.  A sector still
 *              rotating after max_sweeps fails the update with MPS_E_NOCONV
 *              before any state changes.
 *   jacobi_tol rotate a vector pair while |<x,y>| > tol * |x| |y|; <= 0
 *              means max(vector length, 64) * 2^-52.  The SVD of an r x c
 *              sector orthogonalises its min(r, c) rows or columns.
 *   form       MPS_FORM_PLAIN_C128 (default): every step in complex128.
 *              MPS_FORM_SPLIT_BF16X3: the charge-triple products of Theta
 *              formation run on the matrix cores with each operand split into
 *              three BF16 parts (x = hi + mid + lo, 2^-24 relative) and the
 *              eight BF16 part products other than lo*lo per real product,
 *              the leading one and the corrections accumulated apart in FP32
 *              within 32-wide k chunks, the chunks summed in FP64 (FP32
 *              accuracy: about 2^-24 per product plus the FP32 rounding of
 *              the chunk sums); the gate mix, the Jacobi
 *              SVD, the cut and the update stay FP64, and the site tensors
 *              are stored in complex128.
 *   modulus    0 (default): U(1), the charge of Eqs. (E2)-(E4) is the particle
 *              number.  n >= 2: a discrete Abelian charge Z_n (the paper's
 *              general Abelian symmetries, Sec. I), the particle number mod n,
 *              with d <= n (every local occupation a distinct charge): bond
 *              charges lie in 0..n-1, the charge balance of Eq. (E4) holds mod
 *              n (bond 0 carries n_photons mod n), and a left/right charge
 *              pair of a site is allowed when (cL - cR) mod n is an occupation
 *              (with d == n every pair; with d < n a sector's rows and columns
 *              are the charges within d of its middle charge, cyclically).  A
 *              Z_n state takes dense gates only (mps_apply_layer_dense).
 * The kept count is K = max(1, min(chi_max, K_eps, K_zero)). */
typedef enum { MPS_FORM_PLAIN_C128 = 0, MPS_FORM_SPLIT_BF16X3 = 1 } mps_form;

typedef struct {
  int chi_max;
  double cutoff;
  double zero_tol;
  int max_sweeps;
  double jacobi_tol;
  int form;                    /* mps_form */
  int modulus;                 /* 0: U(1), the charge is the particle number;
                                  n >= 2: Z_n, the particle number mod n
                                  (requires d <= n; bond charges 0..n-1) */
  int blocked_sweeps;          /* blocked Jacobi sweeps before the scalar
                                  finish (0: the default, 32); at most
                                  max_sweeps.  A diagnostic: a small value
                                  sends sectors through the scalar sweeps. */
  int select_scratch;          /* 1: the cut's sort always goes through
                                  device memory, as it does when a gate has
                                  more than 4096 candidate values (0: LDS
                                  when it fits).  A diagnostic. */
  int sweep_graph;             /* 1: the step launches of a Jacobi sweep are
                                  captured once per update call into a HIP
                                  graph (on the handle's stream, thread-local
                                  capture) and the graph is launched once per
                                  sweep; 0 (default): launched one by one.
                                  Results are identical either way. */
  int tile_tuning;             /* split-BF16 form: 1 (default): the output tile
                                  of the sector products is chosen per batch by
                                  a tuner keyed on the histogram of charge-block
                                  sizes (the first batch with a key times every
                                  shape once; the choice is kept for the
                                  process); 0: always 64 x 64; 2..5: always
                                  shape 0..3 (64x64, 32x64, 64x32, 32x32; a
                                  diagnostic).  The products are bitwise the
                                  same for every shape. */
  int jacobi_block;            /* vectors per block of the blocked Jacobi SVD:
                                  8 or 16, or 0 (default): chosen per update
                                  call, 8 when the longest vector has 320 or
                                  more elements and the call has fewer pairs
                                  of 16-vector blocks than twice the GPU's
                                  compute units, else 16.  A block pair of 2b
                                  vectors is orthogonalised per visit through
                                  its 2b x 2b Gram matrix; smaller blocks make
                                  shorter visits and more of them.  In a batch
                                  the first state's value serves every state. */
  int jacobi_lockstep;         /* 0 (default): each sector of an update sweeps
                                  at its own pace -- step launch t runs every
                                  sector's own next round-robin step, and a
                                  sector with few blocks starts its next sweep
                                  while the largest one is still in its first;
                                  1: all sectors sweep in lockstep, a sweep
                                  lasting as many launches as the largest
                                  sector has steps.  The same visits in the
                                  same order per sector either way, so the
                                  same results bit for bit.  Lockstep is also
                                  used with sweep_graph and for sectors of
                                  more than 4224 vectors (blocks of 8) or 2176
                                  (blocks of 16).  In a batch the first
                                  state's value serves every state. */
} mps_opts;

/* Per-handle counters, accumulated since creation or mps_reset_stats.
 * *_ms are kernel times from HIP events on the handle's stream; they are
 * filled only while timing is enabled (mps_set_timing).  Flop figures are
 * algorithmic: 8*nL*nM*nR per charge triple for Theta formation; for the
 * blocked Jacobi step kernel 8*nv^2*len per block-pair Gram matrix formed and
 * 8*nv^2*len per block pair rotated (nv vectors of length len = max(r, c);
 * plus the c x c accumulator of a tall sector); 8*r*c*K per sector for the
 * update product. */
typedef struct {
  long long gates;             /* two-site updates applied                    */
  long long layers;            /* layers (apply calls touching this state)    */
  long long sectors;           /* Theta(m) sectors decomposed                 */
  long long sweeps;            /* Jacobi sweeps summed over sectors           */
  long long rotations;         /* Jacobi block pairs rotated                  */
  double theta_flops, jacobi_flops, update_flops;
  double theta_ms, jacobi_ms, jacobi_aux_ms, select_ms, update_ms;
  long long theta_launches, jacobi_launches, jacobi_aux_launches, select_launches,
      update_launches;
  long long polish_launches;   /* batches that needed the scalar Jacobi finish */
  double max_discarded;        /* largest per-gate discarded weight            */
  double min_margin;           /* smallest (s_{K-1} - s_K)/s_0 at a cut        */
  double gemm_ms;              /* split-BF16 form: the charge-triple products  */
  long long gemm_launches;     /*   (theta_ms then covers the gate mix)        */
  double gemm_mfma_flops;      /* split-BF16 form: flops the BF16 matrix-core  */
                               /*   products execute, tile padding included    */
                               /*   (64 per complex multiply-add: 4 real       */
                               /*   products x 8 split terms x 2)              */
  double split_ms;             /* split-BF16 form: splitting the site tensors  */
                               /*   into BF16 planes before the products       */
  double leak_total;           /* weight removed by the local cutoff, summed   */
                               /*   over gates (see mps_last_leaks)            */
  long long graph_launches;    /* sweeps launched as a captured graph          */
  double host_plan_ms;         /* host wall time spent planning updates (the   */
                               /*   charge-sector work lists, uploads packed,  */
                               /*   update lists from the kept counts); always */
                               /*   measured                                   */
  long long tile_tunings;      /* split form: batches that timed every tile    */
                               /*   shape of the products (new histogram key)  */
  int gemm_variant;            /* split form: tile shape of the last products  */
                               /*   launch: 0 64x64, 1 32x64, 2 64x32, 3 32x32 */
  int jacobi_block;            /* vectors per Jacobi block of the last update  */
                               /*   (8 or 16; see mps_opts.jacobi_block)       */
  double jacobi8_ms, jacobi8_flops;  /* the share of jacobi_ms, jacobi_flops */
  long long jacobi8_launches;  /*   and jacobi_launches from updates that used */
                               /*   blocks of 8 (jacobi_block_step8)           */
} mps_stats;

/* Fill *o with the defaults: chi_max 0, cutoff 0, zero_tol 1e-13,
 * max_sweeps 40, jacobi_tol 0, plain form, modulus 0, blocked_sweeps 0,
 * select_scratch 0, sweep_graph 0, tile_tuning 1, jacobi_block 0,
 * jacobi_lockstep 0. */
void mps_default_opts(mps_opts* o);

/* Create a state of L sites with local dimension d (occupations 0..d-1,
 * Eq. (E1)) and n_photons = N photons.
 *   bond_dim[L+1]    dimension of every bond; bond_dim[0] = bond_dim[L] = 1.
 *   bond_charge[]    right-charges (Eq. (E3)) of every bond index, bonds 0..L
 *                    concatenated (sum of bond_dim entries); bond 0 is {N}
 *                    and bond L is {0} (Eq. (E4)); every charge in [0, N].
 *   gamma            NULL, or L host pointers; gamma[s] is the Vidal tensor
 *                    Gamma[s] as a bond_dim[s] x bond_dim[s+1] row-major
 *                    complex matrix in the caller's index order; entries
 *                    whose charge difference lies outside 0..d-1 must be 0.
 *   lambda           NULL, or L+1 host pointers to the Schmidt values of
 *                    every bond (bond 0 and L: {1}).  Required with gamma.
 * With gamma == NULL every bond must have dimension 1 and the state is the
 * Fock product state whose occupations are the charge differences.
 * Bond indices are reordered internally by ascending charge (stable).
 * Errors: MPS_E_ARG, MPS_E_CHARGE, MPS_E_NOMEM, MPS_E_DEVICE. */
mps_status mps_create(int L, int d, int n_photons, const int* bond_dim,
                      const int* bond_charge, const mps_z* const* gamma,
                      const double* const* lambda, const mps_opts* opts,
                      const mps_device* dev, mps_t* out);

/* Convenience: the Fock product state |occupation[0], ..., occupation[L-1]>. */
mps_status mps_create_product(int L, int d, const int* occupation,
                              const mps_opts* opts, const mps_device* dev,
                              mps_t* out);

/* A product state whose local states carry one or two independent U(1)
 * charges (the paper's general Abelian symmetries, Sec. I; for example two
 * species of hard-core bosons, local state p = 2 a + b carrying the pair of
 * species numbers (a, b)).  charge_map[p * ncomp + k] (0..64) is component k
 * of the charge of local state p; ncomp is 1 or 2, the rows must be distinct,
 * and the modulus option must be 0.  The right-charges of Eq. (E3) are then
 * sums of these (pairs for ncomp = 2), the rule of Eq. (E2) allows an entry
 * on local state p between left charge cL and right charge cR when
 * cL - cR = charge_map[p], and a gate must conserve the charge of the pair
 * of sites: such a state takes dense gates only (mps_apply_layer_dense, which
 * refuses a charge-changing element).  Amplitudes, norms, sampling and the
 * cut are those of the U(1) case; mps_bond_charges reads the bookkeeping as
 * components, mps_bond_sectors as internal integer keys.
 * Errors: MPS_E_ARG, MPS_E_NOMEM, MPS_E_DEVICE. */
mps_status mps_create_product_charges(int L, int d, const int* occupation, int ncomp,
                                      const int* charge_map, const mps_opts* opts,
                                      const mps_device* dev, mps_t* out);

/* Number of charge components of the state (1 for U(1) and Z_n states, 1 or
 * 2 for mps_create_product_charges). */
mps_status mps_charge_components(mps_t h, int* ncomp);


/* Release every resource of the handle (NULL is accepted). */
mps_status mps_destroy(mps_t h);

/* One two-site update on sites (site, site+1): Theta formation by charge-
 * sector-matched products, the gate applied block by block per total local
 * photon number n (its elements are those of the symmetric power of u2,
 * projected to occupations < d), per-middle-charge SVD, one cut over all
 * sectors, and the new site tensors, Schmidt values and bond charges.
 *   discarded  out, may be NULL: sum of the dropped squared singular values.
 * Errors: MPS_E_ARG, MPS_E_NOCONV, MPS_E_NUMERIC, MPS_E_NOMEM, MPS_E_DEVICE. */
mps_status mps_apply_gate(mps_t h, int site, const mps_z u2[4], double* discarded);

/* The same update for ngates gates on pairwise disjoint site pairs
 * (|site_i - site_j| >= 2), executed together: one launch per step for all
 * of them.  u2s holds ngates 2x2 matrices back to back; discarded[ngates]
 * (may be NULL) receives each gate's weight.  The result equals applying the
 * gates one by one in any order. */
mps_status mps_apply_layer(mps_t h, int ngates, const int* sites,
                           const mps_z* u2s, double* discarded);

/* The same layer for gates given as dense two-site matrices, such as the
 * Trotter factors exp(-i dt h) of a Hamiltonian with [H, N] = 0 (Sec. II:
 * Bose-Hubbard, XXZ with the magnetisation as the charge).  g4s holds
 * ngates matrices of d^2 x d^2 complex elements back to back, each
 * row-major with row index p*d + q (occupations of sites site and site+1
 * after the gate) and column index a*d + b (before).  The library reads
 * the blocks G^(n)[p][a] = g4[(p, n-p), (a, n-a)] and the rest of the
 * update is that of mps_apply_layer.  Elements with p + q != a + b must
 * vanish (for a Z_n state: p + q != a + b mod n, and the blocks are indexed
 * by the total mod n): those up to 1e-13 times the gate's largest element
 * modulus are dropped, a larger one fails with MPS_E_CHARGE before any state
 * changes.
 * Errors: as mps_apply_layer; MPS_E_CHARGE as above. */
mps_status mps_apply_layer_dense(mps_t h, int ngates, const int* sites,
                                 const mps_z* g4s, double* discarded);

/* Batching form: one layer of each of nh independent states (different
 * circuits, sizes and cut options, one local dimension d, one stream),
 * executed together -- the updates of all states share every launch, so
 * the device holds many independent sectors at once (the paper's
 * independent two-site updates, Sec. II, across circuits).  State i takes
 * ngates[i] gates (0 allowed) on pairwise disjoint site pairs; sites and u2s
 * hold the gates of all states back to back in state order, as does
 * discarded (may be NULL).  hs[0]'s workspaces and its max_sweeps and
 * jacobi_tol serve the batch; each state keeps its own chi_max, cutoff and
 * zero_tol.  The result for each state equals mps_apply_layer on it alone.
 * If any update fails no state changes.  A state may appear once.
 * Errors: as mps_apply_layer; MPS_E_ARG for mixed d, forms or streams. */
mps_status mps_apply_batch(int nh, const mps_t* hs, const int* ngates,
                           const int* sites, const mps_z* u2s, double* discarded);

/* Re-truncate bond `bond` (1..L-1) from its stored Schmidt values with the
 * same rule (chi_max, cutoff, the handle's zero_tol), without an SVD: the
 * dropped Schmidt vectors are removed from sites bond-1 and bond.  Exact
 * when the state is in canonical form.  discarded may be NULL. */
mps_status mps_truncate(mps_t h, int bond, int chi_max, double cutoff,
                        double* discarded);

/* Amplitudes c_{i_1..i_L} (Eq. (E2)) of `count` occupation patterns,
 * occ[count*L] row-major; out[count].  A pattern whose photon number differs
 * from N, with an occupation outside 0..d-1, or whose charge path meets a
 * charge absent from a bond gives exactly 0. */
mps_status mps_amplitude(mps_t h, int count, const int* occ, mps_z* out);

/* <psi|psi> by full contraction of the transfer matrices (not sum lambda^2). */
mps_status mps_norm(mps_t h, double* norm2);

/* mps_norm for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same contraction and kernels, with the environment buffers and the work
 * lists in a fixed device array of the library (64 MiB per GPU, held until the
 * process ends) instead of the handle's growable workspaces.  Allocates no
 * device or pinned memory.  The result equals mps_norm's.
 * Limit: (2 + d) * chi^2 * 16 bytes plus the work lists must fit in 64 MiB,
 * chi the largest bond dimension (d = 4: chi up to about 830); a larger state
 * fails with MPS_E_ARG before any device work.  Runs on the GPU current when
 * the handle was created and on its stream, and returns after its device work
 * has finished.  All calls share one array per GPU (its contents are those of
 * the last call); calls are serialised by a lock inside the library, so calls
 * from several host threads do not overlap on the device.
 * Errors: MPS_E_ARG, MPS_E_DEVICE. */
mps_status mps_norm_noalloc(mps_t h, double* norm2);

/* Exact samples of output patterns (the read-out of a boson-sampling
 * circuit, Sec. I): pattern i is drawn with probability |c_i|^2 / <psi|psi>,
 * c_i as in Eq. (E2), by the chain rule from mode L-1 down to mode 0.  Mode
 * k of sample j takes the smallest occupation whose cumulative conditional
 * probability exceeds uniforms[j*L + k] (caller-supplied, each in [0, 1);
 * the library draws no random numbers).
 *   occ    out, count*L row-major occupations;
 *   prob   out, may be NULL: |c_i|^2 / <psi|psi> of each drawn pattern.
 * All samples advance together, one mode per round; the samples on one
 * charge share the products with that charge's blocks, and each round is
 * planned on the device (the host waits once per call).  Bonds may carry at
 * most 1024 charges.  The left
 * environments of every bond (as many complex entries as the squared bond
 * dimensions, summed: about the size of the state) and the rounds' buffers
 * (about 10 vectors of the largest charge block per sample, at most 8192
 * samples at a time) are held in device memory during the call only.
 * Errors: MPS_E_ARG (a uniform outside [0, 1), more than 1024 charges on a
 * bond), MPS_E_NUMERIC (a vanished or non-finite marginal; occ and prob are
 * then undefined), MPS_E_NOMEM, MPS_E_DEVICE. */
mps_status mps_sample(mps_t h, int count, const double* uniforms, int* occ, double* prob);

/* Bookkeeping of bond `bond` (0..L): its distinct charges in ascending
 * order and their multiplicities.  cap is the capacity of charge[] and
 * count[]; *nsec receives the number of sectors (MPS_E_ARG if > cap). */
mps_status mps_bond_sectors(mps_t h, int bond, int cap, int* nsec,
                            int* charge, int* count);

/* Bookkeeping of bond `bond` with the charges as components: sector i has
 * charge comps[i * ncomp .. i * ncomp + ncomp - 1] (ncomp from
 * mps_charge_components; sectors in lexicographic order) and multiplicity
 * count[i].  cap is the number of sectors comps[] and count[] can hold. */
mps_status mps_bond_charges(mps_t h, int bond, int cap, int* nsec, int* comps, int* count);

/* Schmidt values of bond `bond`, ordered by ascending charge and, within a
 * charge, descending value.  *n receives the bond dimension. */
mps_status mps_bond_lambda(mps_t h, int bond, int cap, int* n, double* lambda);

/* Copy site tensor B[site] = Gamma[site] lambda[site+1] as a dense
 * rows x cols row-major matrix (rows: bond `site`, cols: bond `site`+1, both
 * in ascending-charge order).  cap is out's capacity in elements. */
mps_status mps_site_tensor(mps_t h, int site, size_t cap, int* rows, int* cols,
                           mps_z* out);

/* Per-gate weight removed by the local cutoff in the last apply call that
 * touched h (its gates in call order): |lambda_s theta~|^2 of the two-site
 * tensor before the gate minus |theta|^2 after it.  With d <= N the gate
 * the MPS applies is the two-mode gate projected to occupations < d, which is
 * not unitary on the blocks of total photon number n >= d (Sec. II gives d as
 * the local dimension); this is the weight that projection removes, apart
 * from the SVD's discarded weight.  cap is the capacity of leak; *n receives
 * the gate count (MPS_E_ARG if above cap). */
mps_status mps_last_leaks(mps_t h, int cap, int* n, double* leak);

/* Enable (1) or disable (0) HIP-event timing of every kernel launch. */
mps_status mps_set_timing(mps_t h, int on);
mps_status mps_get_stats(mps_t h, mps_stats* s);
mps_status mps_reset_stats(mps_t h);

/* Wait for all work of the handle; reports deferred device errors. */
mps_status mps_sync(mps_t h);

/* Thread-local text of the last error (never NULL). */
const char* mps_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* U1MPS_H */
