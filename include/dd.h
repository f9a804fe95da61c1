/*
 * dd.h - C ABI of the MI355X direct domain-decomposition (DD) FEM solver.
 *
 * Method (Moshfegh & Vouvakis, "Direct Solution of FEM Models: Are Sparse
 * Direct Solvers the Best Strategy?", section II): a decomposed FEM problem
 * with primal DoFs inside every domain and dual DoFs (Lagrange multipliers) on
 * the interfaces forms the arrowhead system
 *
 *      [ blkdiag(K_i)  B^T ] [ u      ]   [ f ]
 *      [ B             0   ] [ lambda ] = [ 0 ]
 *
 * with complex-symmetric domain matrices K_i (K_i = K_i^T, not Hermitian) and
 * a signed Boolean interface operator B.  The solver
 *   1. eliminates the primal DoFs of every domain by independent sparse LDL^T
 *      factorisations (multifrontal, batched across domains on the GPU),
 *   2. forms each domain's dual interface block B_i K_i^-1 B_i^T,
 *   3. assembles and factors the block-sparse symmetric auxiliary matrix
 *      F = sum_i B_i K_i^-1 B_i^T with a block LDL^T using restricted
 *      Bunch-Kaufman pivoting (symbolic phase on the clique graph of the
 *      domains), and
 *   4. recovers the primal unknowns for many right-hand sides by independent
 *      forward/backward substitutions u_i = K_i^-1 (f_i - B_i^T lambda).
 *
 * Threading: a context may be used by one host thread at a time.  Every entry
 * point returns a dd_status and never throws; the message of the last failure
 * of the calling thread is returned by dd_last_error().
 *
 * Memory: the library never allocates device memory.  The caller allocates a
 * device workspace of dd_workspace_size() bytes (for example a torch uint8
 * tensor) and binds it with dd_bind_workspace().  Host state is owned by the
 * context and released by dd_destroy().
 */
#ifndef DD_H
#define DD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* One complex FP64 value; layout-compatible with std::complex<double>,
 * C99 double _Complex and torch.complex128. */
typedef struct { double re, im; } dd_z;

typedef struct dd_ctx_s *dd_ctx;

typedef enum {
    DD_OK = 0,
    DD_ERR_ARG = -1,           /* null pointer, negative size, bad option            */
    DD_ERR_PATTERN = -2,       /* malformed CSR pattern                              */
    DD_ERR_MAP = -3,           /* malformed interface map                            */
    DD_ERR_STATE = -4,         /* call out of order (e.g. solve before factor)       */
    DD_ERR_NOMEM = -5,         /* workspace too small / host allocation failed       */
    DD_ERR_SINGULAR = -6,      /* a pivot block had to be perturbed: the domain (or
                                  auxiliary) matrix is singular to working
                                  precision inside a pivot tile (dd_info says
                                  where)                                          */
    DD_ERR_NUMERIC = -7,       /* non-finite pivot in the factorisation, or a
                                  non-finite refinement residual                  */
    DD_ERR_NOT_CONVERGED = -8, /* refinement hit refine_maxit above refine_tol      */
    DD_ERR_DEVICE = -9         /* a HIP runtime call failed                          */
} dd_status;

enum { DD_FP64 = 0, DD_FP32_REFINE = 1 };

/* Front-size buckets of the Schur-update tile policy: fronts of size
 * [0,512), [512,1024), [1024,2048), [2048,4096), [4096,...). */
#define DD_TILE_BUCKETS 5

/* Sparsity pattern of one domain matrix K_i (host memory).
 * Square n x n, CSR, 0-based, both triangles stored (structurally symmetric),
 * column indices strictly increasing within a row, every diagonal present. */
typedef struct {
    int32_t n;
    int64_t nnz;
    const int64_t *rowptr;   /* [n+1], rowptr[0] = 0, rowptr[n] = nnz */
    const int32_t *colind;   /* [nnz] */
} dd_pattern;

/* The decomposed problem (host memory; deep-copied by dd_setup).
 * Interface map: the entries of domain i are [imap_ptr[i], imap_ptr[i+1]);
 * entry e says row imap_mult[e] of B has value imap_sign[e] (+1 or -1) in
 * column imap_dof[e] of domain i.  Every multiplier id in [0, n_mult) must
 * appear in exactly two entries, belonging to two different domains. */
typedef struct {
    int32_t n_dom;
    const dd_pattern *dom;     /* [n_dom] */
    int64_t n_mult;
    const int64_t *imap_ptr;   /* [n_dom+1] */
    const int32_t *imap_dof;   /* [imap_ptr[n_dom]] local dof in the domain   */
    const int64_t *imap_mult;  /* [imap_ptr[n_dom]] multiplier id             */
    const int8_t  *imap_sign;  /* [imap_ptr[n_dom]] +1 / -1                    */
    const float   *dof_xyz;    /* optional [sum n_i][3] coordinates that steer
                                  the nested-dissection orderings (any embedding,
                                  e.g. logical lattice positions); may be NULL,
                                  then a graph-only ordering is used            */
} dd_problem;

typedef struct {
    int32_t precision;     /* DD_FP64, or DD_FP32_REFINE: complex FP32 fronts,
                              Schur updates and substitutions, FP64 pivot blocks,
                              FP64 residuals and refinement updates             */
    double  refine_tol;    /* DD_FP32_REFINE: stop when every column has both
                              residuals relative to its right-hand side at or
                              below refine_tol (default 1e-9): the torn one,
                              [f - K u - B^T lam; -B u], and the assembled one,
                              f - A u~ with A = sum_i R_i^T K_i R_i and u~ every
                              DoF's lowest-numbered copy (the residual of the
                              undecomposed FEM system)                         */
    int32_t refine_maxit;  /* DD_FP32_REFINE: iteration cap (default 20)        */
    int32_t max_rhs;       /* columns per internal solve block; the workspace is
                              sized for it, larger nrhs are solved in blocks
                              (default 64)                                       */
    int32_t leaf_size;     /* nested-dissection leaf size (default 48)          */
    int32_t use_graph;     /* 1: capture the factorisation (per value pointer)
                              and the solve core (per column count) into
                              hipGraphs on first use and replay them; 2: the
                              solve core only; 0: plain launches.  Timed
                              kernels always run plain.                       */
    int32_t verbose;       /* print the symbolic summary to stderr              */
    int32_t schur_tile[DD_TILE_BUCKETS];
                           /* output tile edge of the trailing Schur update per
                              front-size bucket: 64 or 128 (0 = library default:
                              64 below 1024, 128 above); dd_tune measures it  */
    int32_t verify_schedule;
                           /* 1: dd_setup (and dd_tune's re-plan) also checks
                              on the host that the factorisation's launches on
                              its side streams never touch data that an
                              unordered launch writes, and that fronts alive
                              at the same time do not share memory
                              (DD_ERR_STATE if they do); costs host time   */
    const char *tune_cache;/* optional path of dd_tune's tile cache (a text
                              file, one line per problem shape and device:
                              key and the five tile edges); dd_tune reads its
                              line instead of measuring, or appends one after
                              measuring.  Copied by dd_setup; NULL: none    */
} dd_options;

typedef struct {
    double  t_setup;        /* host seconds in dd_setup                         */
    double  t_factor;       /* device seconds of the last dd_factor             */
    double  t_solve;        /* device seconds of the last dd_solve              */
    double  flops_factor;   /* algorithmic real flops of one factorisation
                               (complex FMA = 8), from the symbolic structure   */
    double  flops_solve;    /* algorithmic real flops of one solve per RHS      */
    double  bytes_factor;   /* bytes of the stored factors (L panels + inverse
                               interface blocks) in the factor precision        */
    int64_t workspace_bytes;
    int32_t n_fronts_domain;
    int32_t n_fronts_aux;
    int32_t max_front_aux;
    int32_t max_front_domain;
    int32_t refine_iters;   /* refinement iterations of the last dd_solve       */
    double  rel_resid;      /* refined solves: max over columns of the assembled
                               residual ||f - A u~|| / ||f|| (see refine_tol)   */
    int32_t n_perturbed;    /* pivots perturbed in the last dd_factor           */
    int32_t numeric_flags;  /* nonzero if a non-finite pivot was met            */
    double  bytes_solve;    /* bytes of stored factors one solve of one column
                               block reads (forward and backward sweeps)        */
    double  rel_resid_torn; /* refined solves: max over columns of the torn
                               residual ||[f - K u - B^T lam; -B u]|| / ||f||   */
    int32_t bad_domain;     /* lowest domain with a perturbed or non-finite
                               pivot, n_dom for the auxiliary matrix, -1 none   */
    int32_t n_pivot_2x2;    /* 2 x 2 pivots chosen by the last dd_factor        */
    int32_t n_interchanges; /* pivot interchanges inside the pivot tiles         */
    int32_t tuned_from_cache; /* 1 if the last dd_tune took its tiles from the
                               tune_cache file                                   */
} dd_info;

/* Defaults listed above. */
void dd_default_options(dd_options *opt);

/* Symbolic phase, host only (no GPU call).  Section II: the decomposed
 * problem has primal DoFs in the domains and dual DoFs on the interfaces; the
 * domains are eliminated by independent sparse direct factorisations, and the
 * auxiliary matrix is factored after a symbolic step on the clique graph of
 * its block-wise sparse structure.  Here: validates the problem, orders every
 * domain by nested dissection with its interface DoFs last, builds the
 * multifrontal trees, groups the multipliers into blocks with identical domain
 * pairs, orders the block (clique) graph of the auxiliary matrix, and plans the
 * workspace and every launch.  opt may be NULL (defaults).
 * Errors: DD_ERR_ARG, DD_ERR_PATTERN, DD_ERR_MAP, DD_ERR_NOMEM. */
dd_status dd_setup(const dd_problem *prob, const dd_options *opt, dd_ctx *out);

/* Bytes of device workspace the context needs (host only). */
dd_status dd_workspace_size(dd_ctx ctx, int64_t *bytes);

/* Binds caller-owned device memory (>= dd_workspace_size bytes, 256-byte
 * aligned) and uploads the static index tables into it (synchronous copy on
 * the current device).  The memory must stay allocated until dd_destroy or
 * the next bind.  Errors: DD_ERR_NOMEM (too small), DD_ERR_DEVICE. */
dd_status dd_bind_workspace(dd_ctx ctx, void *dev_ptr, int64_t bytes);

/* Capacity of the static workspace array of dd_bind_static_workspace. */
#define DD_STATIC_WORKSPACE_BYTES (128LL << 20)

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): binds the library's
 * own static device array of DD_STATIC_WORKSPACE_BYTES (one per GPU, held
 * until the process ends) as the workspace of ctx, on the current device,
 * instead of caller memory.  Calls no allocating routine: it uploads the
 * index tables (synchronous copy) and nothing else; the context's events and
 * streams are created by its first dd_factor.  Problems whose
 * dd_workspace_size exceeds the capacity are refused with DD_ERR_NOMEM.
 * The array is shared by every context bound to it on that GPU and holds
 * the tables and factors of the context bound last: binding another
 * context invalidates the previous one (its later calls return
 * DD_ERR_STATE), and work of two contexts on one GPU's array must not
 * overlap.  Nothing in it needs clearing: every call writes what it reads.
 * Errors: DD_ERR_ARG, DD_ERR_NOMEM, DD_ERR_DEVICE. */
dd_status dd_bind_static_workspace(dd_ctx ctx);

/* Numeric factorisation (section II: the primal DoFs of every domain are
 * eliminated by independent sparse LDL^T factorisations, leaving the dual
 * blocks B_i K_i^-1 B_i^T; their sum, the symmetric block-wise sparse
 * auxiliary matrix, is factored by a block LDL^T with restricted
 * Bunch-Kaufman pivoting), enqueued on hip_stream (a hipStream_t; NULL = the
 * null stream).  vals: device array of the values of all domain matrices
 * concatenated in domain order, nnz_i each in the CSR order of dd_setup's
 * patterns.  The values are read during the call's stream work only (FP32
 * mode keeps an FP64 copy in the workspace for refinement).
 * Returns after enqueueing.  Numerical problems are reported by dd_get_info
 * and by the next dd_solve / dd_solve_subset, which waits for the
 * factorisation to finish and reads its status words: a non-finite pivot
 * gives DD_ERR_NUMERIC (nothing is solved); perturbed pivots give
 * DD_ERR_SINGULAR in FP64 mode (the solution of the perturbed factors is
 * still written) and in FP32_REFINE mode only when the refinement does not
 * reach refine_tol. */
dd_status dd_factor(dd_ctx ctx, const dd_z *vals, void *hip_stream);

/* Solves the arrowhead system for nrhs right-hand sides (section II: the
 * condensed right-hand side gives the multipliers through the factored
 * auxiliary matrix, then the primal unknowns of every domain are recovered by
 * independent forward/backward substitutions; section III: many
 * excitations).
 * f: device, torn right-hand sides, column-major with leading dimension ldf
 *    >= sum n_i; rows of domain i start at sum_{j<i} n_j.
 * u: device output in the same layout (ldu >= sum n_i); may not alias f.
 * lam: optional device output of the multipliers, n_mult x nrhs column-major
 *    with leading dimension ldl >= n_mult (NULL to skip).
 * FP32 mode refines in FP64 until refine_tol (DD_ERR_NOT_CONVERGED if the cap
 * is hit; u and lam still hold the last iterate).  FP64 mode is asynchronous
 * on hip_stream apart from the status check: the first solve after a
 * dd_factor waits for the factorisation to finish (see dd_factor for the
 * codes).  FP32 mode synchronises the stream once per refinement step. */
dd_status dd_solve(dd_ctx ctx, int32_t nrhs, const dd_z *f, int64_t ldf, dd_z *u,
                   int64_t ldu, dd_z *lam, int64_t ldl, void *hip_stream);

/* Solve with recovery of a subset of the primal unknowns (section II: after
 * the multipliers, the primal unknowns of all domains or of only some are
 * recovered by independent substitutions).  Same arguments and layouts as
 * dd_solve without the multipliers; domain_mask is a host array of n_dom
 * bytes.  The condensation and the auxiliary solve involve every domain;
 * only the domains with domain_mask[i] != 0 are back-substituted, and only
 * their rows of u are written (the other rows are left unchanged).  Those
 * rows equal dd_solve's bit for bit.  The mask is copied during the call
 * (stream-ordered).  FP64 contexts only: refinement needs every domain's
 * solution (DD_ERR_ARG for FP32_REFINE).
 * Errors: DD_ERR_ARG, DD_ERR_STATE (not factored), DD_ERR_DEVICE. */
dd_status dd_solve_subset(dd_ctx ctx, int32_t nrhs, const dd_z *f, int64_t ldf, dd_z *u, int64_t ldu,
                          const uint8_t *domain_mask, void *hip_stream);

/* Recovery of selected primal unknowns only (section II: all or a subset of
 * the primal unknowns are recovered; here at the granularity of single DoFs,
 * e.g. observation points).  rows: host array of nsel torn row ids (the
 * torn layout of dd_solve: rows of domain i start at sum_{j<i} n_j); only
 * the domains holding them are back-substituted, and out (device, nsel x
 * nrhs column-major, leading dimension ldo >= nsel) receives u at those
 * rows, equal bit for bit to dd_solve's.  f as in dd_solve.  Synchronises
 * hip_stream before returning.  FP64 contexts only.
 * Errors: DD_ERR_ARG (bad row, sizes, FP32_REFINE), DD_ERR_STATE,
 * DD_ERR_DEVICE. */
dd_status dd_solve_dofs(dd_ctx ctx, int32_t nrhs, const dd_z *f, int64_t ldf, int64_t nsel, const int64_t *rows,
                        dd_z *out, int64_t ldo, void *hip_stream);

/* Statistics; synchronises the streams of the last factor/solve. */
dd_status dd_get_info(dd_ctx ctx, dd_info *info);

/* Interface DoFs of domain dom in the order used by dd_get_interface_inverse
 * (ascending local dof).  dofs may be NULL to query the count only. */
dd_status dd_get_interface_dofs(dd_ctx ctx, int32_t dom, int32_t *count, int32_t *dofs);

/* Copies (K_dom^-1) restricted to the interface DoFs, i.e. the inverse of the
 * interface Schur complement, as a dense count x count column-major complex
 * FP64 matrix into device memory out (after dd_factor, stream-ordered). */
dd_status dd_get_interface_inverse(dd_ctx ctx, int32_t dom, dd_z *out, void *hip_stream);

/* Algorithmic factorisation flops of one domain (its fronts and the inverse
 * of its interface block), from the symbolic structure (host only). */
dd_status dd_get_domain_flops(dd_ctx ctx, int32_t dom, double *flops);

/* Diagnostics: device timing of one factorisation kernel.  After
 * dd_kernel_timer_start(ctx, kernel) every launch of that kernel by the
 * following dd_factor calls is bracketed by a pair of events on its stream
 * (up to 4096 launches).  dd_kernel_timer_read synchronises and returns the
 * summed device seconds, the number of launches and their algorithmic flops.
 * kernel = DD_KERNEL_NONE stops timing. */
enum {
    DD_KERNEL_NONE = -1,
    DD_KERNEL_SCHUR_UPDATE = 0,   /* trailing update A22 -= L21 (L21 D)^T (MFMA)   */
    DD_KERNEL_PANEL_SOLVE = 1,    /* L21 D = A21 P^T L11^-T, L21 (MFMA)            */
    DD_KERNEL_PIVOT_TILE = 2,     /* restricted Bunch-Kaufman tile factorisation
                                     of the first tile of each outer block       */
    DD_KERNEL_INVERSE_UPDATE = 3, /* interface inverse X = Z^T D^-1 Z (MFMA)      */
    DD_KERNEL_COLUMN_UPDATE = 4   /* the outer block's later tiles: columns
                                     A(:, t) -= L W^T by its earlier tiles (MFMA)
                                     and the pivot tile, in one launch           */
};
dd_status dd_kernel_timer_start(dd_ctx ctx, int32_t kernel);
dd_status dd_kernel_timer_read(dd_ctx ctx, double *seconds, int64_t *launches, double *flops);

/* Tile autotuner for the batched factorisation of uneven fronts (section II
 * builds the method on many independent dense operations, to expose
 * concurrency for parallel and GPU processing).  With a tune_cache whose
 * line matches this problem's front shapes, precision and device, its tiles
 * are used without measuring.  Otherwise, for every front-size bucket
 * that has fronts, times the first
 * outer block's Schur update of all its fronts with 64 x 64 and 128 x 128
 * tiles on the bound workspace (a few launches each, events on hip_stream),
 * keeps the faster one, re-plans the launch sequences with that policy and
 * uploads them.  The workspace layout is unchanged.  schur_tile (may be NULL)
 * receives the chosen edges, DD_TILE_BUCKETS entries (0 for empty buckets);
 * pass them in dd_options.schur_tile to skip tuning next time.  Overwrites
 * workspace contents: call it before dd_factor (a previous factorisation is
 * discarded).  Synchronises hip_stream.
 * Errors: DD_ERR_STATE (no workspace), DD_ERR_DEVICE. */
dd_status dd_tune(dd_ctx ctx, int32_t *schur_tile, void *hip_stream);
/* (The cache line is appended after the measurement; a cache file that
 * cannot be read or written is ignored.) */

/* Releases the context (host state only; the workspace stays caller-owned). */
void dd_destroy(dd_ctx ctx);

/* Message of the last failed call on this thread ("" if none). */
const char *dd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DD_H */
