/*
 * hinqs.h -- C ABI of the MI355X (gfx950) selected-CI subspace solver.
 *
 * The library builds the second-quantized Hamiltonian
 *     H = E_core + sum_pq h_pq a+_p a_q + 1/2 sum_pqrs g_pqrs a+_p a+_q a_s a_r
 * (paper Sec. 2.2, the Hamiltonian stated before Step 1; E_core is the
 * constant the paper calls E_nuc) restricted to a sampled determinant set B,
 * [H_B]_ij = <x_i|H|x_j> (Sec. 2.2, Step 3), applies it to blocks of vectors
 * and finds its lowest eigenpair with a Davidson eigensolver (Step 3), which
 * yields E_0 and Psi_0 as a linear combination of the determinants of B.
 * Around that solve it provides the selection steps of the same section:
 * the classical expansion of B (Eq. 2), PT2 scores of candidates (Eq. 3),
 * stable top-k ranking, incremental updates of B with the growth rules of
 * Step 2, the product-space closure of B, and the spin-marginal teacher
 * weights of Psi_0 (Step 4, Eqs. 5-6).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - A determinant is a pair of occupation strings (alpha, beta), each a
 *   uint64 whose bit p is set when spatial orbital p is occupied with that
 *   spin (Sec. 2.1: x = (sigma_alpha, sigma_beta)).  norb <= 32.
 * - Fermionic sign gauge: |x> = prod_{P occupied, ascending} a+_P |vac>, with
 *   the alpha spin-orbitals 0..norb-1 ordered before the beta ones.
 * - Two-electron integrals are passed in chemists' notation (pq|rs), i.e.
 *   g_pqrs of the Hamiltonian above equals (pr|qs).
 * - Vectors indexed by determinant follow the caller's order of
 *   hinqs_set_determinants unless HINQS_SORTED_ORDER is given.  Blocks of k
 *   vectors are ndet x k row-major (the k values of one determinant are
 *   contiguous).
 * - Every call is issued on the stream given to hinqs_create.  Device
 *   pointers must be valid on the context's device.  Calls that return
 *   host results (energies, statistics) synchronize that stream.
 * - Status: 0 on success, a negative HINQS_E_* code otherwise; the message
 *   of the last failure is available from hinqs_last_error.  A context is
 *   not thread-safe; concurrent calls on one context are undefined.
 */
#ifndef HINQS_H
#define HINQS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define HINQS_OK                   0
#define HINQS_E_INVALID_ARG       -1   /* bad pointer, size or option */
#define HINQS_E_NOT_READY         -2   /* integrals or determinants not set */
#define HINQS_E_ASYMMETRIC        -3   /* h or (pq|rs) lack real-orbital symmetry */
#define HINQS_E_BAD_OCCUPATION    -4   /* wrong electron count or bits >= norb */
#define HINQS_E_DUPLICATE         -5   /* a determinant appears twice */
#define HINQS_E_UNSUPPORTED       -6   /* norb > 32, unsupported block size */
#define HINQS_E_NOT_CONVERGED     -7   /* outputs hold the best estimate */
#define HINQS_E_NONFINITE         -8   /* NaN or Inf in the inputs */
#define HINQS_E_OOM               -9   /* device allocation failed */
#define HINQS_E_HIP              -10   /* a HIP runtime call failed */

/* arithmetic of sigma products */
#define HINQS_FP64   0
#define HINQS_FP32   1
/* Davidson precision modes */
#define HINQS_SOLVE_FP64   0   /* every sigma product in FP64 */
#define HINQS_SOLVE_MIXED  1   /* FP32 sigma until the residual is below mixed_switch or stalls near
                                  the FP32 rounding floor, then FP64 refinement */

/* flags */
#define HINQS_SORTED_ORDER 1   /* vectors are in the library's internal sorted order */
#define HINQS_AUTOTUNE     2   /* hinqs_opts.flags: tune the sigma launch shape before solving */
#define HINQS_NO_GRAPH     4   /* hinqs_opts.flags, batched solves: launch each kernel directly */
#define HINQS_LARGEST      8   /* hinqs_top_k: select the largest values instead of the smallest */

/* hinqs_grow_basis modes */
#define HINQS_GROW_APPEND   0   /* append the K best candidates, then cap the set at b_max */
#define HINQS_GROW_REBUILD  1   /* keep the K best of the set and the candidates together */

/* excitation classes stored in a coupling descriptor (bits 0..2) */
#define HINQS_EXC_1A   1   /* single, alpha */
#define HINQS_EXC_1B   2   /* single, beta */
#define HINQS_EXC_2AA  3   /* double, both alpha */
#define HINQS_EXC_2BB  4   /* double, both beta */
#define HINQS_EXC_2AB  5   /* double, one alpha and one beta */

typedef struct hinqs_ctx hinqs_ctx;

typedef struct hinqs_opts {
    int    block;          /* Davidson block size k in {1,2,4,8,16}; default 8 */
    int    max_space;      /* largest subspace before a thick restart, in [3*block, 96]; default 6*block */
    int    max_iter;       /* iteration cap; default 200 */
    double tol;            /* stop when ||H c - E c||_2 <= tol for the lowest root; default 1e-8 */
    int    precision;      /* HINQS_SOLVE_FP64 or HINQS_SOLVE_MIXED; default FP64 */
    double precond_floor;  /* |theta - H_ii| is clamped below at this value; default 1e-8 */
    double mixed_switch;   /* MIXED: switch to FP64 once the residual is below this; default 1e-5 */
    int    flags;          /* HINQS_SORTED_ORDER for guess and coeffs; HINQS_AUTOTUNE */
} hinqs_opts;

typedef struct hinqs_stats {
    int    iterations;         /* Davidson iterations (all precisions) */
    int    iterations_fp32;    /* of which with FP32 sigma products */
    int    sigma_blocks;       /* block sigma products applied */
    int    sigma_columns;      /* vectors those products carried (<= block each) */
    int    restarts;
    double residual;           /* final ||r||_2 of the lowest root */
    double ms_total;           /* wall time of the call */
    double ms_sigma;           /* time inside sigma kernels (HIP events) */
    int64_t nnz;               /* stored off-diagonal couplings */
    int    second_passes;      /* iterations whose projection against the basis needed a second
                                  pass (a new direction kept < 1/2 of its norm in the first) */
} hinqs_stats;

typedef struct hinqs_info {
    int     norb, nalpha, nbeta;
    int64_t ndet;
    int64_t nnz;               /* off-diagonal couplings stored in the sparse H_B */
    int32_t n_alpha_strings;   /* distinct alpha strings in B */
    int32_t n_beta_strings;    /* distinct beta strings in B */
    int64_t device_bytes;      /* device memory held by the context */
    double  ms_sort;           /* last set_determinants: sort + string tables */
    double  ms_connect;        /* last set_determinants: coupling enumeration */
    double  ms_elements;       /* last element build (Slater-Condon) */
} hinqs_info;

typedef struct hinqs_batch_stats {
    int     instances;
    int     converged;         /* instances whose lowest root reached tol */
    int     iterations;        /* batched iterations (one graph launch each) */
    int     graphs;            /* graphs captured (one per subspace size); 0 with HINQS_NO_GRAPH */
    double  ms_total;          /* wall time of the call */
    double  ms_setup;          /* merge, buffers, initial block, graph capture */
    double  ms_iterations;     /* the iteration loop without capture */
    double  max_residual;      /* largest final ||r||_2 of a lowest root */
    int64_t ndet;              /* determinants over all instances */
    int64_t nnz;               /* stored couplings over all instances */
    int     sigma_team, sigma_unroll, sigma_occupancy;  /* sigma launch shape used */
    double  sigma_elements;    /* H x products applied: sum over instances of (nnz + ndet) * block per sigma */
    int     chunk_rows;        /* rows per chunk of the tall-skinny kernels */
    int     rr_threads;        /* threads of the per-instance Rayleigh-Ritz kernel */
    double  ms_tune;           /* time spent timing launch shapes (HINQS_AUTOTUNE, first call per size class) */
} hinqs_batch_stats;

/* Fill *opts with the defaults listed above. */
void hinqs_opts_default(hinqs_opts *opts);

/*
 * Device memory of a context.  Every buffer the library keeps (the sorted
 * determinant tables, couplings, matrix elements, the Davidson basis, and the
 * staging of calls that work in sorted order) comes from `alloc` and goes back
 * through `free`, both called with the context's stream and the `user` pointer
 * given to hinqs_create; a framework passes its own caching allocator here so
 * the library's workspace shares its memory pool.  alloc returns NULL when it
 * cannot provide `bytes` (the call then fails with HINQS_E_OOM and leaves the
 * context usable); free receives only pointers alloc returned, with the same
 * stream.  Buffers are released by hinqs_destroy, and when a larger one
 * replaces them.
 */
typedef void *(*hinqs_alloc_fn)(size_t bytes, void *hip_stream, void *user);
typedef void (*hinqs_free_fn)(void *ptr, void *hip_stream, void *user);

/*
 * Create a context bound to HIP device `device` and stream `hip_stream`
 * (a hipStream_t; NULL = the null stream).  *out receives the handle.
 * alloc_fn / free_fn: the device allocator (both NULL: hipMalloc / hipFree;
 * exactly one NULL is INVALID_ARG); user is passed back to them unchanged.
 * Errors: INVALID_ARG, OOM, HIP.
 */
int hinqs_create(hinqs_ctx **out, int device, void *hip_stream, hinqs_alloc_fn alloc_fn,
                 hinqs_free_fn free_fn, void *user);

/* Release every device buffer of the context (through its free_fn).  NULL is ignored. */
void hinqs_destroy(hinqs_ctx *ctx);

/* Message of the last failure on ctx ("" if none); valid until the next call. */
const char *hinqs_last_error(const hinqs_ctx *ctx);

/*
 * Load the Hamiltonian of Sec. 2.2.
 *   h      host, norb*norb doubles, row-major, symmetric (|h_pq - h_qp| <= 1e-12 max|h|)
 *   eri    host, norb^4 doubles, row-major chemists' (pq|rs), 8-fold symmetric
 *          (real orbitals) to 1e-12 of its largest magnitude
 *   e_core constant energy (nuclear repulsion / frozen core), added on the diagonal
 * The inputs are copied; the caller may free them on return.  If determinants
 * are already set, the matrix elements are rebuilt (couplings are kept).
 * Errors: INVALID_ARG (norb < 1), UNSUPPORTED (norb > 32), NONFINITE,
 * ASYMMETRIC, OOM, HIP.  norb must equal that of the determinants if set.
 */
int hinqs_set_integrals(hinqs_ctx *ctx, int norb, const double *h, const double *eri,
                        double e_core);

/*
 * Load the determinant set B (Sec. 2.2, Steps 1-3: the sampled basis).
 *   alpha, beta  host, ndet uint64 strings each, any order (the caller order)
 *   nalpha, nbeta electrons per spin; every string must have exactly that many
 *                 bits set, all below norb
 * The library sorts B, builds its string tables and enumerates every coupled
 * pair (excitation degree 1 or 2) with its fermionic sign; if integrals are
 * set it also evaluates the matrix elements.  Requires hinqs_set_integrals
 * first (for norb).  Inputs are copied.
 * Errors: NOT_READY (no integrals), INVALID_ARG (ndet < 1, nalpha/nbeta out of
 * range), BAD_OCCUPATION, DUPLICATE, OOM, HIP.
 */
int hinqs_set_determinants(hinqs_ctx *ctx, int64_t ndet, const uint64_t *alpha,
                           const uint64_t *beta, int nalpha, int nbeta);

/*
 * As hinqs_set_determinants, with alpha and beta already in device memory
 * (ndet uint64 each, on the context's device); validation runs on the GPU.
 * The arrays are copied; the caller keeps ownership.
 * Errors: as hinqs_set_determinants.
 */
int hinqs_set_determinants_device(hinqs_ctx *ctx, int64_t ndet, const uint64_t *alpha,
                                  const uint64_t *beta, int nalpha, int nbeta);

/*
 * Block sigma product S = H_B X (the repeated operation of the Davidson
 * iteration of Step 3).
 *   k          number of vectors, 1 <= k <= 16
 *   X          device, ndet x k row-major, doubles (FP64) or floats (FP32)
 *   S          device, same shape and type; must not overlap X
 *   precision  HINQS_FP64 or HINQS_FP32 (FP32 values, vectors and sums)
 *   flags      HINQS_SORTED_ORDER: X and S are in internal sorted order
 * Unless X and S are in sorted order, 16-byte aligned and k is 1, 2, 4, 8 or
 * 16, the call stages them through sorted-order blocks of ndet x K values
 * (K = k rounded up to those sizes) held by the context.
 * Errors: NOT_READY, INVALID_ARG, UNSUPPORTED, OOM (staging), HIP.
 */
int hinqs_sigma(hinqs_ctx *ctx, int k, const void *X, void *S, int precision, int flags);

/*
 * hinqs_sigma for callers that cannot allocate device memory: code under HIP
 * graph capture, allocation-free serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, result and errors as hinqs_sigma; it calls no
 * allocator, no memset and no synchronisation, and the caller still provides
 * X and S.  The sigma row counters and, when staging is needed (see
 * hinqs_sigma), the two ndet x K staging blocks live in one static device
 * array of HINQS_NOALLOC_SCRATCH_BYTES per GPU, set up by the first
 * hinqs_create on that GPU and held until the process ends.  A call needing
 * more than the array (4096 + 2 * ndet * K * element size bytes when staged)
 * fails with UNSUPPORTED.  Every call on one GPU shares that GPU's array and
 * finds the previous call's contents there: calls that overlap on one GPU
 * (other streams, contexts or threads) race and must be serialised by the
 * caller.
 */
#define HINQS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int hinqs_sigma_noalloc(hinqs_ctx *ctx, int k, const void *X, void *S, int precision, int flags);

/*
 * Lowest eigenpair of H_B by block Davidson (Step 3, warm-startable as the
 * paper's incremental backend is).
 *   opts    NULL for defaults
 *   guess   device, ndet doubles or NULL; used as the first trial vector
 *   energy  host, receives E_0 (including e_core)
 *   coeffs  device, ndet doubles, receives Psi_0 normalized to 1 with its
 *           largest-magnitude component positive
 *   stats   host or NULL
 * Errors: NOT_READY, INVALID_ARG, NOT_CONVERGED (energy/coeffs hold the last
 * Ritz pair), OOM, HIP.
 */
int hinqs_lowest_eigenpair(hinqs_ctx *ctx, const hinqs_opts *opts, const double *guess,
                           double *energy, double *coeffs, hinqs_stats *stats);

/*
 * One- and two-particle density matrices of the vector c (not renormalized):
 *   rdm1[p,q]     = sum_s   <c| a+_{p s} a_{q s} |c>                (device, norb^2)
 *   rdm2[p,q,r,s] = sum_st  <c| a+_{p s} a+_{r t} a_{s t} a_{q s} |c> (device, norb^4)
 * so that E = e_core + sum h rdm1 + 1/2 sum (pq|rs) rdm2 for a normalized
 * eigenvector.  These are the derivatives of the energy with respect to the
 * integrals (Hellmann-Feynman), the gradient signal behind the autograd
 * binding.  Accumulation uses floating-point atomics, so results are
 * reproducible to rounding only.
 * Errors: NOT_READY, INVALID_ARG, OOM, HIP.
 */
int hinqs_rdm12(hinqs_ctx *ctx, const double *coeffs, double *rdm1, double *rdm2, int flags);

/*
 * Energy gradient with respect to symmetric integrals for a normalized
 * eigenvector c:  grad_h = scale * (rdm1 + rdm1^T)/2 and
 * grad_eri = scale * 1/2 * (average of rdm2 over the 8 index permutations of
 * real-orbital symmetry).  A perturbation that keeps the integrals symmetric
 * changes E by sum(grad_h * dh) + sum(grad_eri * deri) to first order.
 *   grad_h   device, norb^2;  grad_eri device, norb^4
 * Errors: as hinqs_rdm12.
 */
int hinqs_integral_grad(hinqs_ctx *ctx, const double *coeffs, double scale, double *grad_h,
                        double *grad_eri, int flags);

/* Diagonal H_ii (device, ndet doubles). */
int hinqs_diag(hinqs_ctx *ctx, double *diag, int flags);

/*
 * Export the couplings in caller order: for caller row i, entries
 * rowptr[i]..rowptr[i+1]-1 of col (caller index j) and desc.  Pass NULL for
 * col/desc to only fill rowptr (device, ndet+1 int64).  col (int32) and desc
 * (uint32) are device arrays of nnz entries; entries within a row are in an
 * unspecified order.  desc layout: bits 0-2 excitation class (HINQS_EXC_*),
 * bit 3 sign (1 = negative), bits 4-8 h1, 9-13 h2, 14-18 p1, 19-23 p2
 * (spatial orbitals; holes are occupied in x_j, particles in x_i; same-spin
 * doubles have h1<h2 and p1<p2; for HINQS_EXC_2AB h1/p1 are alpha and h2/p2
 * beta; singles leave h2 = p2 = 0).  The sign is that of the operator string
 * a+_p a_h (single), a+_p1 a+_p2 a_h2 a_h1 (double) applied to |x_j>.
 */
int hinqs_connectivity(hinqs_ctx *ctx, int64_t *rowptr, int32_t *col, uint32_t *desc);

/* Sorted position -> caller index (device, ndet int32). */
int hinqs_permutation(hinqs_ctx *ctx, int32_t *perm);

/*
 * Tall-skinny Gram product G = A^T B, the Rayleigh-Ritz projection kernel of
 * the Davidson solver (FP64 matrix cores, fixed-order reduction):
 *   A  device, nrows x ma row-major with leading dimension lda >= ma
 *   B  device, nrows x nb row-major with leading dimension ldb >= nb
 *   G  device, ma x nb row-major
 * Needs no integrals or determinants.  ma <= 96, nb <= 16.
 * Errors: INVALID_ARG, UNSUPPORTED, OOM, HIP.
 */
int hinqs_gram(hinqs_ctx *ctx, int64_t nrows, const double *A, int lda, int ma, const double *B,
               int ldb, int nb, double *G);

/*
 * Pick the launch shape of the block-sigma kernel (workgroup team width,
 * software-pipeline depth, workgroups per CU) for blocks of k vectors in
 * `precision` (HINQS_FP64 / HINQS_FP32) on the current Hamiltonian, by
 * timing each candidate on the device; later sigma products of that k and
 * precision use it.  Results are cached per process by device architecture,
 * k, precision and problem-size class (and in the text file named by the
 * environment variable HINQS_TUNE_CACHE, when set), so a second call on a
 * similar problem costs no device time.  shape (host, may be NULL) receives
 * {team, unroll, workgroups per CU}; *ms (may be NULL) the tuned launch time
 * in milliseconds.  Sigma results do not depend on the shape.
 * Errors: NOT_READY, INVALID_ARG, OOM, HIP.
 */
int hinqs_autotune(hinqs_ctx *ctx, int k, int precision, int *shape, double *ms);

/* Sizes and timings of the current state. */
int hinqs_get_info(hinqs_ctx *ctx, hinqs_info *info);

/*
 * Batched instances.  A context also holds a list of independent instances
 * (for example the points of a bond-length scan: each its own norb, electron
 * counts, integrals and determinant set, as for hinqs_set_integrals and
 * hinqs_set_determinants), solved together for their lowest eigenpairs
 * (paper Sec. 2.2, Step 3, once per instance).  The batch does not touch
 * the context's single determinant set.
 *
 * hinqs_batch_clear drops every instance.
 *
 * hinqs_batch_add copies one instance from host memory (same arguments and
 * validation as hinqs_set_integrals + hinqs_set_determinants, errors
 * likewise) and builds its couplings and matrix elements.  *index (may be
 * NULL) receives its position in the batch.
 *
 * hinqs_batch_info: *ninst instances; offsets (host, ninst + 1, may be NULL)
 * receives the first coefficient of each instance in the concatenated
 * vector (offsets[ninst] = total determinants); *nnz (may be NULL) the
 * stored couplings over all instances.
 *
 * hinqs_batch_lowest_eigenpair solves all instances with FP64 block Davidson
 * (opts as for hinqs_lowest_eigenpair; precision must be HINQS_SOLVE_FP64;
 * max_space is capped at 64 and rounded down to a multiple of block, and
 * must be at least 3 * block; every instance needs at least max_space
 * determinants).  All instances advance together and each iteration is one
 * replay of a captured hipGraph (HINQS_NO_GRAPH: plain launches, same
 * arithmetic); converged instances are skipped from then on.  Outputs:
 * energies (host, ninst), coeffs (device, total determinants; instance i at
 * offsets[i], in its own caller order unless HINQS_SORTED_ORDER), status
 * (host, ninst, may be NULL: 0 or HINQS_E_NOT_CONVERGED), iterations (host,
 * ninst, may be NULL), stats (may be NULL).  Returns NOT_CONVERGED when any
 * instance missed the tolerance (outputs hold the best estimates).
 * Errors: NOT_READY (empty batch), UNSUPPORTED, INVALID_ARG, OOM, HIP.
 */
int hinqs_batch_clear(hinqs_ctx *ctx);
int hinqs_batch_add(hinqs_ctx *ctx, int norb, const double *h, const double *eri, double e_core,
                    int64_t ndet, const uint64_t *alpha, const uint64_t *beta, int nalpha, int nbeta,
                    int *index);
int hinqs_batch_info(hinqs_ctx *ctx, int *ninst, int64_t *offsets, int64_t *nnz);
int hinqs_batch_lowest_eigenpair(hinqs_ctx *ctx, const hinqs_opts *opts, double *energies,
                                 double *coeffs, int *status, int *iterations,
                                 hinqs_batch_stats *stats);

/*
 * Classical expansion of the determinant set (paper Sec. 2.2, Eq. 2): the
 * ntop determinants of B with the largest |c_i| are chosen (ties: the lower
 * index first; ntop is clamped to ndet), and every determinant y outside B
 * with <y|H|x> != 0 for at least one chosen x is returned once, in ascending
 * (alpha, beta) order (alpha compared first).  A connection is an element
 * whose computed Slater-Condon value is not exactly zero; every single and
 * double excitation of x is examined, so the result holds at most
 * ntop * (singles + doubles per determinant) entries.
 *   coeffs     device, ndet doubles (caller order unless HINQS_SORTED_ORDER);
 *              NaN or Inf gives NONFINITE
 *   ntop       >= 1
 *   capacity   entries available in out_alpha / out_beta (>= 0); the first
 *              min(capacity, *count) determinants are written
 *   out_alpha, out_beta  device, capacity uint64 each (may be NULL when
 *              capacity is 0)
 *   count      host, receives the number of distinct determinants found
 *   top        device, ntop int32, or NULL: the chosen determinants, largest
 *              |c| first (caller indices, or sorted positions with
 *              HINQS_SORTED_ORDER)
 * Device scratch of about 12 bytes per determinant of B plus 20 bytes per
 * examined excitation is allocated for the call.  Needs integrals and
 * determinants.
 * Errors: NOT_READY, INVALID_ARG, NONFINITE, UNSUPPORTED (2^31 or more
 * examined excitations: expand fewer determinants per call), OOM, HIP.
 */
int hinqs_expand(hinqs_ctx *ctx, const double *coeffs, int64_t ntop, int64_t capacity,
                 uint64_t *out_alpha, uint64_t *out_beta, int64_t *count, int32_t *top, int flags);

/*
 * Second-order (Epstein-Nesbet) importance of candidate determinants
 * (paper Sec. 2.2, Eq. 3) against Psi_0 = sum_i c_i |x_i> over B:
 *   numer[t] = sum_i c_i <x_t|H|x_i>   (the diagonal term is included when
 *                                      x_t lies in B)
 *   hxx[t]   = <x_t|H|x_t>            (including e_core)
 *   score[t] = numer[t]^2 / |e0 - hxx[t]|   (IEEE division: inf when
 *                                      e0 == hxx[t] and numer != 0)
 *   coeffs     device, ndet doubles (caller order unless HINQS_SORTED_ORDER)
 *   e0         the reference energy E_0 (finite)
 *   cand_alpha, cand_beta  device, ncand uint64 each; any determinants with
 *              the electron counts of B (duplicates and members of B allowed)
 *   numer, hxx, score      device, ncand doubles each, or NULL to skip
 * Sums are in an unspecified but fixed order (bitwise reproducible on one
 * device).  A candidate with bits at or above norb or the wrong electron
 * count gets NaN outputs and the call returns BAD_OCCUPATION after the
 * others are written.
 * Errors: NOT_READY, INVALID_ARG, NONFINITE, BAD_OCCUPATION, OOM, HIP.
 */
int hinqs_pt2(hinqs_ctx *ctx, const double *coeffs, double e0, int64_t ncand,
              const uint64_t *cand_alpha, const uint64_t *cand_beta, double *numer, double *hxx,
              double *score, int flags);

/*
 * hinqs_pt2 for the candidates x = the determinants of B themselves (their
 * eviction ranking in Sec. 2.2, Step 2), from the coupling matrix: numer is
 * the row of H_B c, diagonal included (one sigma product), hxx the diagonal,
 * score = numer^2 / |e0 - hxx|.  Equal to hinqs_pt2 on B's own strings up to
 * the order of the sums.
 *   coeffs            device, ndet doubles (caller order unless HINQS_SORTED_ORDER)
 *   numer, hxx, score device, ndet doubles each (same order), or NULL to skip
 * Errors: NOT_READY, INVALID_ARG, NONFINITE, OOM, HIP.
 */
int hinqs_pt2_members(hinqs_ctx *ctx, const double *coeffs, double e0, double *numer, double *hxx,
                      double *score, int flags);

/*
 * Stable selection of the k smallest (or, with HINQS_LARGEST, the k
 * largest) of n doubles: idx (device, k int32) receives their indices in
 * that order, ties broken by the lower index; -0.0 equals +0.0.  This is the
 * ranking of Sec. 2.2: the cold start keeps the candidates of lowest H_xx,
 * later iterations the candidates of highest PT2 score (Eq. 3).
 *   values  device, n doubles; NaN gives NONFINITE
 * Needs no integrals or determinants.  Allocates about 12 n bytes of device
 * scratch for the call.
 * Errors: INVALID_ARG (k < 1, k > n), UNSUPPORTED (n >= 2^31), NONFINITE,
 * OOM, HIP.
 */
int hinqs_top_k(hinqs_ctx *ctx, int64_t n, const double *values, int64_t k, int flags, int32_t *idx);

/*
 * Spin-marginal teacher weights of a vector over B (paper Sec. 2.2, Step 4,
 * Eqs. 5-6):
 *   p_alpha(s) = sum of c_x^2 over the x in B with alpha string s
 *   p_beta(s)  = sum of c_x^2 over the x in B with beta string s
 *   weights[x] = p_alpha(alpha_x) p_beta(beta_x) / Z,  Z = the sum over B
 *                of those products, so the weights sum to 1
 *   coeffs   device, ndet doubles (caller order unless HINQS_SORTED_ORDER)
 *   weights  device, ndet doubles (same order), or NULL
 *   p_alpha  device, n_alpha_strings doubles indexed like the ascending
 *            distinct alpha strings of hinqs_distinct_strings, or NULL
 *   p_beta   device, n_beta_strings doubles, likewise, or NULL
 * Sums run in a fixed order (bitwise reproducible).  The weights keep no
 * phase and no alpha-beta correlation of c, as the factorized target does.
 * Errors: NOT_READY (no determinants), INVALID_ARG (all coefficients zero),
 * NONFINITE, OOM, HIP.
 */
int hinqs_teacher_weights(hinqs_ctx *ctx, const double *coeffs, double *weights, double *p_alpha,
                          double *p_beta, int flags);

/* The distinct alpha and beta strings of B in ascending order (device,
 * n_alpha_strings and n_beta_strings uint64; either may be NULL). */
int hinqs_distinct_strings(hinqs_ctx *ctx, uint64_t *alpha, uint64_t *beta);

/*
 * Incremental update of the determinant set (paper Sec. 2.2: from the second
 * iteration on, Step 2 appends the best-scored new candidates to B and
 * evicts the lowest-scored entries beyond a cap, and Step 3 keeps its state
 * across iterations and warm-starts from the previous eigenvector).
 * The new set B' lists the kept determinants (B without the evicted ones, in
 * their caller order) followed by the appended ones in the given order, and
 * replaces the context's set: afterwards every call sees B' exactly as
 * hinqs_set_determinants would have built it (the same coupled pairs with
 * the same descriptors and values; entries within a row may come in another
 * order, so sigma products agree to rounding).  Couplings between kept
 * determinants are carried over with their values; only pairs that involve
 * an appended determinant are enumerated and evaluated.
 *   n_evict, evict   device, n_evict distinct int32: caller indices of B (or
 *                    sorted positions with HINQS_SORTED_ORDER); may be NULL
 *                    when n_evict is 0
 *   n_add, add_alpha, add_beta  device, n_add uint64 each, determinants not in
 *                    B' otherwise (one that is being evicted may come back);
 *                    may be NULL when n_add is 0
 *   coeffs_old       device, old ndet doubles (old caller order, or old sorted
 *                    order with HINQS_SORTED_ORDER), or NULL
 *   coeffs_new       device, new ndet doubles (new order), or NULL: the warm
 *                    start, coeffs_old on the kept determinants and 0 on the
 *                    appended ones (not renormalized)
 *   ms               host, may be NULL: wall time of the update in ms
 * Device memory for both the old and the new couplings is held during the
 * call.  On INVALID_ARG, BAD_OCCUPATION or DUPLICATE the context is left
 * unchanged; after OOM or HIP it needs hinqs_set_determinants again.
 * Errors: NOT_READY, INVALID_ARG (index out of range or repeated, empty
 * result), BAD_OCCUPATION, DUPLICATE, UNSUPPORTED, OOM, HIP.
 */
int hinqs_update_determinants(hinqs_ctx *ctx, int64_t n_evict, const int32_t *evict, int64_t n_add,
                              const uint64_t *add_alpha, const uint64_t *add_beta, const double *coeffs_old,
                              double *coeffs_new, int flags, double *ms);

/*
 * The basis-update rules of paper Sec. 2.2, Step 2, applied with
 * hinqs_update_determinants (same carried couplings, same warm start):
 *   HINQS_GROW_APPEND (iterations t >= 2): the k candidates of highest score
 *     are appended, highest first; if the set would then exceed b_max
 *     (b_max > 0), the lowest-scored entries of the set and of those k are
 *     dropped until b_max remain.
 *   HINQS_GROW_REBUILD (iteration t = 1): the set becomes the k highest-scored
 *     of the current set and the candidates together, with no cap; kept
 *     members stay in their order, chosen candidates follow, highest first.
 * Ties go to the lower index of the list (current set in caller order, then
 * candidates); -0.0 equals +0.0; NaN scores give NONFINITE.
 *   ncand, cand_alpha, cand_beta, cand_score  device, candidates outside the
 *                    set (uint64 strings, double scores)
 *   k                candidates to append / size of the rebuilt set
 *   basis_score      device, ndet doubles (caller order): required by
 *                    REBUILD, by a capped APPEND and for score_new
 *   b_max            cap (0: none)
 *   coeffs_old/new   as for hinqs_update_determinants (coeffs_new holds at
 *                    least ndet + k doubles)
 *   score_new        device, at least ndet + k doubles, or NULL: the scores of
 *                    the new set in its caller order
 *   ndet_new         host, may be NULL; ms host, may be NULL
 * Errors: as hinqs_top_k and hinqs_update_determinants; INVALID_ARG for a
 * missing basis_score or an unknown mode.
 */
int hinqs_grow_basis(hinqs_ctx *ctx, int mode, int64_t ncand, const uint64_t *cand_alpha,
                     const uint64_t *cand_beta, const double *cand_score, int64_t k,
                     const double *basis_score, int64_t b_max, const double *coeffs_old,
                     double *coeffs_new, double *score_new, int64_t *ndet_new, double *ms);

/* The determinant strings of the current set in caller order (device, ndet
 * uint64 each; either may be NULL). */
int hinqs_get_determinants(hinqs_ctx *ctx, uint64_t *alpha, uint64_t *beta);

/*
 * Product-space closure of the set (the backends named in paper Sec. 2.2,
 * Step 3, diagonalize on the alpha x beta product of the distinct strings of
 * B; this library diagonalizes on B itself): every determinant
 * (a, b) with a among the distinct alpha strings of B and b among its
 * distinct beta strings that is not already in B, in ascending (alpha, beta)
 * order.  *count (host) receives how many there are
 * (n_alpha_strings * n_beta_strings - ndet); the first min(capacity, *count)
 * are written to out_alpha / out_beta (device uint64; may be NULL when
 * capacity is 0).  Appending them with hinqs_update_determinants gives the
 * product space.
 * Errors: NOT_READY, INVALID_ARG, HIP.
 */
int hinqs_product_closure(hinqs_ctx *ctx, int64_t capacity, uint64_t *out_alpha, uint64_t *out_beta,
                          int64_t *count);

/*
 * Host-only helper (no device work): descriptor of the pair x_i <- x_j as
 * the coupling enumerator encodes it, or 0 if the pair differs by more than
 * two electrons or not at all.  Used to check the sign rules on the CPU.
 */
uint32_t hinqs_pair_descriptor(uint64_t alpha_i, uint64_t beta_i, uint64_t alpha_j,
                               uint64_t beta_j);

#ifdef __cplusplus
}
#endif
#endif /* HINQS_H */
