/*
 * qtt.h -- C ABI of libqtt: quantics-tensor-train contraction and rounding
 * on an AMD Instinct MI355X (gfx950).
 *
 * A tensor train (TT) with n cores represents A(i_1..i_n) = C_1(i_1) ... C_n(i_n)
 * (paper Sec. 2, eqs. vector_dec / tensor_dec); core 1 holds the most
 * significant digit (eq. quantization).  Cores cross this boundary as device
 * pointers in row-major layout:
 *     MPS core k: [r_{k-1}, d_k, r_k]           (legs == 1)
 *     MPO core k: [r_{k-1}, d_out, d_in, r_k]   (legs == 2),  y(i) = sum_j A(i,j) x(j)
 * with ranks[0] == ranks[n] == 1.
 *
 * Ownership: the caller owns every device buffer (cores, workspace); the
 * library allocates no device memory after qtt_create.  Host arrays (phys,
 * ranks, info arrays) are caller-owned too.  All work is ordered on the
 * caller's stream.  Calls that return host values (qtt_inner, qtt_round,
 * qtt_orthogonalize, qtt_contract_round, qtt_contract_zipup, qtt_fit)
 * synchronise that stream before returning; qtt_contract, qtt_add and the
 * backward calls do not.
 *
 * Errors: every call returns a qtt_status; QTT_OK == 0, errors are negative.
 * On error the outputs are unspecified and host rank arrays are unchanged.
 * qtt_status_string() names a status.  No C++ exception crosses the ABI.
 */
#ifndef QTT_H_
#define QTT_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QTT_OK = 0,
  QTT_ERR_ARG = -1,         /* null pointer, n < 1, tol < 0, bad enum */
  QTT_ERR_SPEC = -2,        /* unsupported einsum string */
  QTT_ERR_SHAPE = -3,       /* core count / physical size / boundary rank mismatch */
  QTT_ERR_DTYPE = -4,       /* storage type not supported by this call */
  QTT_ERR_WORKSPACE = -5,   /* workspace missing or smaller than required */
  QTT_ERR_NODEVICE = -6,    /* no HIP device, or not a gfx950 device */
  QTT_ERR_HIP = -7,         /* a HIP runtime call failed */
  QTT_ERR_NONFINITE = -8,   /* NaN/Inf met in the data (norm not finite) */
  QTT_ERR_NOCONV = -9,      /* Jacobi sweep cap reached */
  QTT_ERR_UNSUPPORTED = -10 /* size outside the implemented range */
} qtt_status;

/* Storage type of the cores. */
typedef enum { QTT_F64 = 0, QTT_F32 = 1 } qtt_dtype;

/* Arithmetic of the GEMM steps: in a rounding sweep the bond products R C_k
 * of the QR sweep and the products U Sigma = F V that the SVD sweep absorbs
 * into the left neighbour, in qtt_inner_prec the environment products.  The
 * Householder QR, the Jacobi SVD, norms and the rank decisions are always FP64. */
typedef enum {
  QTT_GEMM_FP64 = 0,   /* FP64 MFMA */
  QTT_GEMM_FP32 = 1,   /* operands rounded to FP32, FP32 MFMA accumulation */
  QTT_GEMM_BF16X3 = 2, /* three-piece bf16 split, 3 cross products, FP32 MFMA accumulation */
  QTT_GEMM_BF16X6 = 3  /* three-piece bf16 split, 6 cross products, FP32 MFMA accumulation */
} qtt_prec;

typedef struct {
  int32_t n;             /* number of cores, >= 1 */
  int32_t legs;          /* 1 = MPS (vector), 2 = MPO (matrix) */
  const int32_t *phys;   /* host, n*legs physical sizes (MPO: d_out, d_in per core) */
  int64_t *ranks;        /* host, n+1 bond ranks; rewritten by rounding calls */
  void *const *cores;    /* host array of n device pointers */
  qtt_dtype dtype;
} qtt_tt;

/* Diagnostics of a rounding sweep.  Arrays are caller-owned host buffers of
 * n-1 entries (bond k between cores k and k+1) and may be NULL. */
typedef struct {
  double norm;            /* ||A||_F after the QR sweep */
  double delta;           /* rel_tol * ||A|| / sqrt(n-1) */
  double err_bound;       /* sqrt(sum_k tail_k^2) >= ||A - round(A)||_F */
  double *tail;           /* discarded singular-value 2-norm per bond */
  double *margin_lo;      /* tail(r-1)/delta: > 1 means rank r-1 was not admissible */
  double *margin_hi;      /* tail(r)/delta:  <= 1 unless the max rank capped */
  uint8_t *maxrank_hit;   /* 1 where max_rank capped the bond */
  double *sigma;          /* optional: singular values, bond k at sigma + k*sigma_ld */
  int64_t sigma_ld;       /* row stride of sigma (>= largest pre-truncation rank) */
  int32_t jacobi_sweeps_max;
} qtt_round_info;

typedef struct qtt_context *qtt_handle;

/* Bind a handle to HIP device `device` (must be gfx950). */
int qtt_create(qtt_handle *h, int device);
int qtt_destroy(qtt_handle h);
const char *qtt_status_string(int status);

/* Sweep cap of the one-sided Jacobi SVD used by this handle's rounding,
 * decomposition and batched calls (a batch plan reads it when it is
 * created).  A call whose Jacobi iteration has not reached a sweep without
 * rotations after max_sweeps sweeps returns QTT_ERR_NOCONV; one that
 * reaches it on the last allowed sweep succeeds.  0 restores the default
 * (80); negative values are QTT_ERR_ARG.  Not thread-safe against calls in
 * flight on the same handle. */
int qtt_set_jacobi_max_sweeps(qtt_handle h, int32_t max_sweeps);

/* Operation codes for qtt_workspace_size. */
typedef enum {
  QTT_OP_CONTRACT = 0,
  QTT_OP_ORTHOGONALIZE = 1,
  QTT_OP_ROUND = 2,
  QTT_OP_CONTRACT_ROUND = 3,
  QTT_OP_INNER = 4,
  QTT_OP_INNER_BACKWARD = 5,
  QTT_OP_CONTRACT_BACKWARD = 6
} qtt_op;

/* Device workspace (bytes) needed by `op` on operands a (and b for the binary
 * ops; NULL otherwise).  Pure shape arithmetic: h may be NULL and the core
 * pointers are not dereferenced.  For QTT_OP_CONTRACT_ROUND, spec selects the product
 * and max_rank bounds the result; prec selects the GEMM arithmetic. */
int qtt_workspace_size(qtt_handle h, int op, const char *spec, const qtt_tt *a, const qtt_tt *b,
                       int64_t max_rank, int prec, size_t *bytes);

/* Exact core-by-core Einstein summation (paper Sec. 3.1, eqs. quant_sum and
 * einsum): "i,i->i" (Hadamard, a and b MPS), "ij,j->i" (a an MPO applied to
 * the MPS b) or "ij,jk->ik" (operator product of the MPOs a and b, c an MPO
 * with cores [r, d_out(a), d_in(b), r']).  C_k[(mu,nu), i, (mu',nu')] with
 * the flattened bond xi = mu * r_B + nu.  c's host ranks must equal
 * ranks_a * ranks_b and its cores are caller-allocated; c's dtype must match
 * a's and b's (FP64 or FP32).  An MPO result is rounded by passing it to
 * qtt_round as an MPS of the combined physical size d_out * d_in (same
 * memory).  The fused calls (qtt_contract_round, qtt_contract_zipup) take
 * the two MPS-valued products only.  Asynchronous. */
int qtt_contract(qtt_handle h, const char *spec, const qtt_tt *a, const qtt_tt *b, qtt_tt *c,
                 void *ws, size_t ws_bytes, void *stream);

/* Left-to-right QR sweep (the QR normalisation of Sec. 3.2; canonical form
 * of Sec. 1): cores 1..n-1 become left-orthonormal, the norm moves to core n.
 * In place (FP64 MPS); ranks may shrink to min(d r'_{k-1}, r_k) and are
 * rewritten in t->ranks.  *norm_host receives ||A||_F.  Synchronous. */
int qtt_orthogonalize(qtt_handle h, qtt_tt *t, double *norm_host, void *ws, size_t ws_bytes,
                      void *stream);

/* TT rounding: QR sweep left to right, then truncated SVD sweep right to left
 * (Householder QR and one-sided Jacobi SVD, FP64).  At each bond the kept
 * rank is the smallest r >= 1 whose discarded singular values have 2-norm
 * <= delta = rel_tol * ||A|| / sqrt(n-1), capped at max_rank (<= 0: no cap);
 * this is the truncation of Sec. 3.2's decomposition(max_rank, cutoff)
 * options read as a relative Frobenius tolerance.  In place on an FP64 MPS;
 * the result is right-orthonormal in cores 2..n.  Synchronous. */
int qtt_round(qtt_handle h, qtt_tt *t, double rel_tol, int64_t max_rank, int prec,
              qtt_round_info *info, void *ws, size_t ws_bytes, void *stream);

/* Contraction followed by rounding without materialising the contracted
 * cores: the QR sweep works on the bond products R_{k-1} C_k formed from the
 * operand cores directly (for "ij,j->i": (R X_k) then the MPO core).  out
 * is an FP64 MPS with caller-allocated cores large enough for the rounded
 * ranks (min(r_a r_b, max_rank, profile) per bond is always sufficient);
 * its ranks are written on return.  Synchronous. */
int qtt_contract_round(qtt_handle h, const char *spec, const qtt_tt *a, const qtt_tt *b, qtt_tt *out,
                       double rel_tol, int64_t max_rank, int prec, qtt_round_info *info,
                       void *ws, size_t ws_bytes, void *stream);

/* Stream-ordered qtt_contract_round for HIP graph capture: the same sweeps
 * with no host synchronisation and no host read-back (all rank decisions stay
 * on the device; every launch is sized by the rank bounds, which are the
 * bounds qtt_contract_round's output cores must hold).  On completion of the
 * stream, out's cores hold the rounded train (compact at the rounded ranks),
 * ranks_dev (device, n + 1 int64) the rounded ranks and *status_dev (device)
 * QTT_OK, QTT_ERR_NONFINITE or QTT_ERR_NOCONV.  out's host ranks are not
 * written.  Argument, shape and workspace errors are returned at once, before
 * anything is enqueued.  The workspace is that of qtt_contract_round and must
 * stay untouched until the stream has completed the call.  Asynchronous. */
int qtt_contract_round_async(qtt_handle h, const char *spec, const qtt_tt *a, const qtt_tt *b, qtt_tt *out,
                             double rel_tol, int64_t max_rank, int prec, int64_t *ranks_dev,
                             int32_t *status_dev, void *ws, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * contraction + rounding as qtt_contract_round, with its workspace in a
 * fixed device array of QTT_NOALLOC_SCRATCH_BYTES that the library holds
 * on every device it runs on until the process ends (its address is taken
 * once per device by qtt_create).  Allocates no device memory and calls no
 * allocating routine; the caller still passes the operands and the output
 * cores.  A product whose workspace (qtt_workspace_size, QTT_OP_CONTRACT_ROUND)
 * exceeds the array is rejected with QTT_ERR_WORKSPACE before any launch.
 * Every call on one device shares that device's array: calls that overlap
 * on one device (other host threads, or other streams before this call has
 * returned) race and must not be issued.  Synchronous, like
 * qtt_contract_round. */
#define QTT_NOALLOC_SCRATCH_BYTES (64u << 20)
int qtt_contract_round_noalloc(qtt_handle h, const char *spec, const qtt_tt *a, const qtt_tt *b,
                               qtt_tt *out, double rel_tol, int64_t max_rank, int prec,
                               qtt_round_info *info, void *stream);

/* Decomposition ("zip-up") algorithm of Sec. 3.2 for the same products:
 * copies of both operands are first normalised to the left end (a
 * right-to-left QR sweep, cores 2..n right-orthonormal); a super-core of
 * `ncores` (1 or 2) exact product cores then grows from the left by one
 * bond product S C_k at a time, and whenever it holds ncores cores (and,
 * after the last core, until one remains) its (r d) x (rest) unfolding is
 * split by a truncated one-sided Jacobi SVD: U_r becomes the next result
 * core (left-orthonormal) and Sig_r V_r^T the new super-core.  The kept rank
 * follows qtt_round's rule with delta = rel_tol * ||S||_F / sqrt(n-1), S the
 * super-core being split (the paper's reading of S as the whole result's
 * norm holds only when the exact right part of the product is orthonormal);
 * the contracted train is never formed and never QR-factored as a whole.
 * The result is an approximation whose error is not bounded by
 * info->err_bound in general; its ranks can exceed those of qtt_round.
 * out: FP64 MPS with caller-allocated cores of at least the bounds that
 * qtt_zipup_query returns; its ranks are written on return.  info->norm and
 * info->delta refer to the first split; tail/margins/sigma per bond as for
 * qtt_round.  FP64 operands; prec selects the bond-product arithmetic.
 * Limits: (r d) <= 1024 rows and <= 4096 columns at every split (bounds
 * from qtt_zipup_query), operand unfoldings <= 4096 rows.
 * Synchronous. */
int qtt_contract_zipup(qtt_handle h, const char *spec, const qtt_tt *a, const qtt_tt *b, qtt_tt *out,
                       double rel_tol, int64_t max_rank, int32_t ncores, int prec,
                       qtt_round_info *info, void *ws, size_t ws_bytes, void *stream);

/* Variational fitting of c to the product of a and b ("i,i->i" or
 * "ij,j->i"; paper Sec. 3.3, eq. variational).  The guess c (FP64 MPS,
 * caller-owned cores) is first orthogonalised from the left; then each of
 * `nsweeps` sweeps replaces, from core n down to core 1 and back up to core
 * n, one core at a time by the derivative of <c|a*b> with respect to it
 * (left and right environments of <c|Y> with the exactly contracted product
 * Y formed in the workspace), which is the core minimising ||c - a*b|| when
 * every other core is orthonormal; a QR of the updated core (of its
 * transpose on the way down) keeps the others orthonormal.  Ranks never
 * grow (a QR may shrink one; c->ranks is rewritten).  On return cores 1..n-1
 * are left-orthonormal and *norm_host (nullable) is ||c||.  The result of
 * qtt_contract_zipup is the intended guess.  Synchronous. */
int qtt_fit(qtt_handle h, const char *spec, const qtt_tt *a, const qtt_tt *b, qtt_tt *c, int32_t nsweeps,
            double *norm_host, void *ws, size_t ws_bytes, void *stream);
/* Device workspace (bytes) of qtt_fit; pure shape arithmetic. */
int qtt_fit_workspace_size(const char *spec, const qtt_tt *a, const qtt_tt *b, const qtt_tt *c, size_t *bytes);

/* Variational fitting with super-cores of two adjacent cores (the multi-core
 * strategy of Sec. 3.3; the paper's variational(..., ncores=2)): with the
 * cores left of the pair (q, q+1) left-orthonormal and those right of it
 * right-orthonormal, the pair is replaced by the derivative of <c|a*b> with
 * respect to the fused super-core, S = L_q Y_q Y_{q+1} R_{q+2} (Y the
 * exactly contracted product, formed in the workspace), which is then
 * decomposed again by a truncated SVD (Householder QR + one-sided Jacobi,
 * FP64): the kept rank is the smallest r whose discarded singular values
 * have 2-norm <= rel_tol ||S||_F / sqrt(n-1), capped at max_rank (<= 0: no
 * cap) -- so, unlike qtt_fit, the ranks adapt (grow or shrink).  The guess
 * is first orthogonalised from the left; a sweep runs over the pairs from
 * the right end (core q+1 <- V^T, core q <- U Sigma) and back from the left
 * (core q <- U, core q+1 <- Sigma V^T).  c's cores (FP64, caller-owned) must
 * hold the rank bounds of qtt_fit2_query; c->ranks is rewritten.  info
 * (nullable): norm = ||c||, tail[k] the discarded 2-norm of the last
 * sweep's split at bond k+1, jacobi_sweeps_max; the other fields are not
 * written.  Synchronous. */
int qtt_fit2(qtt_handle h, const char *spec, const qtt_tt *a, const qtt_tt *b, qtt_tt *c, int32_t nsweeps,
             double rel_tol, int64_t max_rank, qtt_round_info *info, void *ws, size_t ws_bytes, void *stream);
/* Linear system W x = b for a symmetric positive definite operator W (FP64
 * MPO with equal input and output sizes; b and the guess x FP64 MPS): the
 * DMRG-like solver of Sec. 5, which minimises the energy
 * J(x) = <x, W x> - 2 <x, b> over one core at a time (ncores = 1, ranks of
 * the guess kept) or over super-cores of two adjacent cores (ncores = 2,
 * the super-core split again by the truncated SVD of qtt_fit2: rel_tol,
 * max_rank, so the ranks adapt).  With the cores outside the block
 * orthonormal the block's minimiser solves the local system
 * A_loc x = b_loc (A_loc from the three-layer environments of <x|W|x>,
 * b_loc from those of <x|b>; symmetric positive definite for such W),
 * solved by a blocked Cholesky factorisation of its lower triangle and two
 * triangular solves (FP64; a pivot that is not positive, i.e. W not SPD,
 * ends in QTT_ERR_NONFINITE).  The guess is orthogonalised from the left
 * first; each of
 * nsweeps sweeps runs from the right end to the left and back.  x's cores
 * are caller-owned with the capacity of qtt_solve_query's bounds (for
 * ncores = 2 a max_rank keeps them small); x->ranks is rewritten.  Limits:
 * local systems of at most 4096 unknowns (rank^2 d^ncores), split rows of
 * at most 1024.  A zero b gives the zero train (all ranks 1) at once.
 * info (nullable): norm = ||x||, jacobi_sweeps_max.  Synchronous. */
int qtt_solve(qtt_handle h, const qtt_tt *w, const qtt_tt *b, qtt_tt *x, int32_t nsweeps, int32_t ncores,
              double rel_tol, int64_t max_rank, qtt_round_info *info, void *ws, size_t ws_bytes, void *stream);
/* Rank capacity (bounds, n+1, nullable) and workspace (bytes) of qtt_solve;
 * pure shape arithmetic. */
int qtt_solve_query(const qtt_tt *w, const qtt_tt *b, const qtt_tt *x, int32_t ncores, int64_t max_rank,
                    int64_t *bounds, size_t *bytes);

/* Linear system W x = b for a symmetric positive definite W by the AMEn
 * solver of Sec. 5 (single-core sweeps with gradient enrichment, after
 * Dolgov and Savostyanov's alternating minimal energy method).  Same
 * operands as qtt_solve, plus z: a train that approximates the residual
 * b - W x (caller-owned FP64 MPS of x's length and sizes; its initial cores
 * are an input, e.g. seeded random numbers; its ranks never grow).  Each
 * step at core q: the one-core local system of qtt_solve gives x_q; its
 * unfolding is truncated by the Jacobi SVD (smallest rank whose discarded
 * singular values have 2-norm <= rel_tol ||x_q||_F / sqrt(n-1), capped at
 * max_rank when > 0); z's core is built from the projection of the
 * residual onto z's frames, and the projection e onto z's frame on one side
 * and x's on the other enriches the kept singular vectors V: the new cores
 * are the orthonormal rows spanning [V^T; e / s] and z's projection / s
 * (Jacobi SVD; directions whose discarded singular values have 2-norm
 * <= 1e-10 are left out, s = ||projected b|| + ||projected W x||), so a
 * bond of x holds up to (truncated rank + z's rank) vectors and no
 * direction in which the residual vanishes (where the frames of x and z
 * overlap near the chain ends a QR would add arbitrary ones; z's end cores
 * are the projections themselves).  x and z are orthogonalised from the
 * left first; each of nsweeps sweeps runs right to left and back.  x's and
 * z's cores are caller-owned with the capacity of qtt_solve_amen_query's
 * bounds (a max_rank keeps x's small); x->ranks and z->ranks are
 * rewritten.  Limits: local systems of at most 4096 unknowns, split rows of
 * at most 1024.  A zero b gives zero trains (all ranks 1) at once.
 * info (nullable): norm = ||x||, jacobi_sweeps_max.  Synchronous. */
int qtt_solve_amen(qtt_handle h, const qtt_tt *w, const qtt_tt *b, qtt_tt *x, qtt_tt *z, int32_t nsweeps,
                   double rel_tol, int64_t max_rank, qtt_round_info *info, void *ws, size_t ws_bytes, void *stream);
/* Rank capacities of x and z (n+1 entries each, nullable) and workspace
 * (bytes) of qtt_solve_amen; pure shape arithmetic. */
int qtt_solve_amen_query(const qtt_tt *w, const qtt_tt *b, const qtt_tt *x, const qtt_tt *z, int64_t max_rank,
                         int64_t *x_bounds, int64_t *z_bounds, size_t *bytes);

/* Rank capacity per bond of qtt_fit2's result (bounds, n+1 entries, nullable:
 * the guess's rank or the largest rank a split can give, whichever is
 * larger) and its device workspace (bytes); pure shape arithmetic. */
int qtt_fit2_query(const char *spec, const qtt_tt *a, const qtt_tt *b, const qtt_tt *c, int64_t max_rank,
                   int64_t *bounds, size_t *bytes);

/* Shape query of qtt_contract_zipup: per-bond rank bounds of the result
 * (n+1 entries, nullable) and the device workspace in bytes (nullable).
 * Pure shape arithmetic; core pointers are not dereferenced. */
int qtt_zipup_query(const char *spec, const qtt_tt *a, const qtt_tt *b, int64_t max_rank, int32_t ncores,
                    int64_t *bounds, size_t *ws_bytes);

/* Exact sum out = sum_t coeffs[t] * terms[t] of `count` (1..16) trains of
 * equal length, legs, physical sizes and dtype (paper Sec. 3.1, addition):
 * core 1 is the row [c_1 X_1 ... c_count X_count], core n the column of the
 * terms' last cores, the others block-diagonal in term order, so out's
 * interior ranks are the sums of the terms' ranks (checked; its cores are
 * caller-allocated).  coeffs may be NULL (all ones).  With one core the
 * result is the weighted sum itself.  Rounding the sum (qtt_round) gives the
 * add-and-truncate of the paper's add().  Asynchronous. */
int qtt_add(qtt_handle h, int32_t count, const qtt_tt *terms, const double *coeffs, qtt_tt *out,
            void *stream);

/* <a, b> = E_n, E_0 = [[1]], E_k = sum_i a_k(i)^T E_{k-1} b_k(i) (the <C|C>
 * contractions of Sec. 3.3).  MPS operands of equal length and physical
 * sizes, FP64 or FP32 (accumulated in the storage type).  Synchronous. */
int qtt_inner(qtt_handle h, const qtt_tt *a, const qtt_tt *b, double *out_host, void *ws,
              size_t ws_bytes, void *stream);
/* qtt_inner with the two GEMMs of every environment step in the arithmetic
 * `prec` (qtt_prec; the precision form of the inner product): FP64 cores
 * only for the reduced forms (QTT_ERR_DTYPE otherwise), same workspace as
 * qtt_inner.  QTT_GEMM_FP64 is qtt_inner.  Synchronous. */
int qtt_inner_prec(qtt_handle h, const qtt_tt *a, const qtt_tt *b, int prec, double *out_host, void *ws,
                   size_t ws_bytes, void *stream);

/* Gradient of g * <a, b> with respect to the cores of a (and of b when db is
 * not NULL): da_k = g * E_{k-1} b_k(i) F_{k+1}^T from left/right environment
 * sweeps (the core derivative of Sec. 3.3, eq. variational).  da/db are
 * caller-allocated MPS with the shapes of a/b.  Asynchronous. */
int qtt_inner_backward(qtt_handle h, const qtt_tt *a, const qtt_tt *b, double g, qtt_tt *da,
                       qtt_tt *db, void *ws, size_t ws_bytes, void *stream);

/* Local backward of qtt_contract: given dC (shaped like c), writes
 * dB_k[nu,j,nu'] = sum_{mu,i,mu'} A_k[mu,i,j,mu'] dC_k[(mu,nu),i,(mu',nu')]
 * (and dA when da is not NULL).  Asynchronous. */
int qtt_contract_backward(qtt_handle h, const char *spec, const qtt_tt *a, const qtt_tt *b,
                          const qtt_tt *dc, qtt_tt *da, qtt_tt *db, void *ws, size_t ws_bytes,
                          void *stream);

/* ---------------------------------------------------------------------------
 * Batched form: `count` independent contract+round problems (arrays a[i],
 * b[i], out[i] of qtt_tt; uneven ranks allowed) in one persistent launch.
 * Each workgroup takes the next problem from a device work queue (largest
 * estimated cost first) and runs the whole QR sweep / Jacobi SVD sweep for
 * it with workgroup-level kernels; rank decisions stay on the device.
 * Bond products and U Sigma = F V run on the bf16 matrix cores: the FP64
 * operands split into three bf16 pieces, six cross products per 32-deep k
 * step accumulated in FP32, the steps added in FP64.  Householder QR, the
 * Jacobi SVD, norms and rank decisions are FP64.  Limits: <= 32 cores per
 * problem, unfolding rows <= 512, Jacobi row length d*r <= 768.
 *
 * qtt_batch_plan_create validates the problems, writes the instance table
 * into ws, picks the GEMM tile shape (64x64, 64x32, 32x64 or 32x32) of each
 * GEMM shape bucket (M > 32, N > 32, K > 64) and a kernel variant (Jacobi
 * block size x grid size) -- when `tune` is non-zero by timing every tile on
 * the bucket's largest shape and every variant on this batch, cached in the
 * file named by QTT_TUNE_CACHE (default ~/.cache/qtt/batched_tune.txt) --
 * and captures the queue reset plus the persistent launch in a hipGraph.
 * qtt_batch_plan_launch replays that graph on `stream` (asynchronous; out
 * cores must stay allocated with room for the rank bounds of each problem).
 * qtt_batch_plan_results synchronises `stream` and writes the rounded ranks
 * of all problems, concatenated (problem i contributes n_i + 1 entries), and
 * optionally the discarded tails (n_i - 1 per problem); it returns
 * QTT_ERR_NONFINITE / QTT_ERR_NOCONV if any problem hit those conditions.
 * The workspace must stay alive and unmodified for the life of the plan.
 * ------------------------------------------------------------------------- */
typedef struct qtt_batch *qtt_batch_plan;
int qtt_batch_workspace_size(qtt_handle h, const char *spec, int32_t count, const qtt_tt *a, const qtt_tt *b,
                             int64_t max_rank, size_t *bytes);
int qtt_batch_plan_create(qtt_handle h, const char *spec, int32_t count, const qtt_tt *a, const qtt_tt *b,
                          qtt_tt *out, double rel_tol, int64_t max_rank, int tune, void *ws, size_t ws_bytes,
                          void *stream, qtt_batch_plan *plan);
int qtt_batch_plan_launch(qtt_batch_plan plan, void *stream);
int qtt_batch_plan_results(qtt_batch_plan plan, int64_t *ranks, double *tails, void *stream);
/* Selected variant (bit 0: Jacobi blocks of 4 rows, bit 1: two workgroups per
 * CU), grid size and the tuning times of the four variants (ms; 0 if the
 * variant came from the cache). */
int qtt_batch_plan_info(qtt_batch_plan plan, int32_t *variant, int32_t *grid, float *tuned_ms);
/* GEMM tile choice of the plan: tiles[8] (0: 64x64, 1: 64x32, 2: 32x64,
 * 3: 32x32) per shape bucket b = (M > 32) + 2 (N > 32) + 4 (K > 64),
 * shapes[8][3] the (M, N, K) the bucket was timed on (zeros: bucket unused),
 * probe_ms[8][4] the median probe time of each tile (zeros: not measured).
 * Any pointer may be NULL. */
int qtt_batch_plan_tiles(qtt_batch_plan plan, uint8_t *tiles, int32_t *shapes, float *probe_ms);
int qtt_batch_plan_destroy(qtt_batch_plan plan);

/* Launch profiling for roofline reports.  qtt_profile_start arms one kernel
 * class (0 = 16-column block-reflector application inside a 64-column
 * block of the Householder QR, 1 = Jacobi SVD, 2 = Householder panel,
 * 3 = V^T Y product of a 64-column block reflector, 4 = its Y += V W
 * update, 5 = Cholesky factor and inverse of a 64 x 64 diagonal block of a
 * solver's local system (with that block's step of the forward
 * substitution), 6 = its trailing update, 7 = the blocked backward
 * triangular solve): every following launch of that class, up to
 * max_launches, is bracketed by HIP events on the stream it is launched on,
 * and its algorithmic bytes and FLOP (from the launch shape) are summed.
 * qtt_profile_stop waits for the last event and returns the launch count,
 * the summed kernel time (ms) and the summed algorithmic bytes / FLOP.  One
 * session per process at a time; not thread-safe.  Allocates HIP events
 * (no device memory). */
int qtt_profile_start(qtt_handle h, int kernel_class, int max_launches);
int qtt_profile_stop(qtt_handle h, int64_t *launches, double *total_ms, double *alg_bytes,
                     double *alg_flops);

#ifdef __cplusplus
}
#endif

#endif /* QTT_H_ */
