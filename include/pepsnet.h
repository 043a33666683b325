/*
 * pepsnet -- Block Belief Propagation (BlockBP) on kagome PEPS, MI355X (gfx950).
 *
 * C ABI of the HIP library libpepsnet.so.  The library computes the BlockBP
 * message update of Eq. blockBP:DefiningEquation: a block of the double-layer
 * (ket x bra) PEPS is contracted with its incoming MPS messages by the
 * boundary-MPS method (Sec. "The boundary-MPS method") and compressed by QR
 * and truncated SVD into outgoing bond-chi MPS messages; sweeps repeat this
 * for every message (Alg. BlockBP_singleBlock for the infinite lattice, the
 * defining equation on finite lattices) and local expectations <S_i . S_j>
 * of the Heisenberg Hamiltonian (Eq. res:afm-h:hamiltonian) are computed from
 * the converged messages.
 *
 * Conventions (part of the ABI):
 *   - complex numbers are interleaved double pairs (re, im), C order;
 *   - a site's ket tensor is t[p][l0][l1][l2][l3], physical dimension d, the
 *     virtual legs ordered by bond angle counter-clockwise from +x
 *     (DL: 0,60,180,240 deg; DR: 0,120,180,300 deg; U: 60,120,240,300 deg);
 *     legs leaving a finite patch have dimension 1;
 *   - tensor order: finite patch -- one tensor per site, sites ordered by
 *     cell (row j outer, column i inner) then U, DL, DR inside a cell;
 *     infinite lattice -- three tensors U, DL, DR (the 3-site unit cell);
 *   - double legs fuse I = ket * D + bra; messages are MPS sites
 *     A[l][I][r], legs in the receiving face's counter-clockwise order.
 * Errors: every call returns BBP_OK (0), a positive warning (outputs valid)
 * or a negative error; pepsnet_last_error() gives the thread-local text.
 * Handles are not thread-safe; a handle owns all of its device memory.
 */
#ifndef PEPSNET_H
#define PEPSNET_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PEPSNET_ABI_VERSION 4

typedef struct pepsnet_s* pepsnet_t;

enum {
  BBP_OK = 0,
  BBP_NOT_CONVERGED = 1, /* warning: max_sweeps reached, outputs valid */
  BBP_PENDING = 2,       /* bbp_server_poll: the request has not finished yet */
  BBP_EINVAL = -1,       /* bad argument; nothing changed */
  BBP_ENOMEM = -2,       /* device allocation failed */
  BBP_EDEVICE = -3,      /* HIP runtime error */
  BBP_ENUMERIC = -4,     /* NaN/Inf or zero trace in a result */
  BBP_EGEOM = -5         /* geometry, tiling or sweep order could not be built */
};

typedef enum { BBP_KAGOME_OPEN = 1, BBP_KAGOME_INF_HEX = 2 } bbp_lattice;
/* arithmetic of the contraction GEMMs (merge, double-layer absorption and
 * the randomized sketches); QR, SVD and normalisation are always FP64 */
typedef enum { BBP_FP64 = 0, BBP_FP32 = 1, BBP_BF16X3 = 2 } bbp_precision;
/* truncated split: T1 exact SVD; T2 randomized range finder (Halko,
 * Martinsson & Tropp 2011, Alg. 4.4) with a SplitMix64 sign sketch */
typedef enum { BBP_SVD_FULL = 0, BBP_SVD_RAND = 1 } bbp_trunc;

typedef struct {
  int32_t abi_version;  /* PEPSNET_ABI_VERSION */
  int32_t lattice;      /* bbp_lattice */
  int32_t Lx, Ly;       /* BBP_KAGOME_OPEN: patch size in unit cells */
  int32_t bLx, bLy;     /* BBP_KAGOME_OPEN: parallelogram block size in cells */
  int32_t hex_N;        /* BBP_KAGOME_INF_HEX: face length N (>= 2), N_T = 3(3N^2-3N+1) */
  int32_t d, D;         /* physical (2) and virtual bond dimension */
  int32_t chi;          /* message bond dimension */
  int32_t chi_env;      /* boundary-chain truncation: chi, or 0 for the exact
                         * contraction of the block (no truncation inside a
                         * message update; the outgoing message is then
                         * compressed to chi by exact truncated SVDs; every
                         * split of the block's chain must then fit the exact
                         * SVD kernels, at most 144 rows and columns after
                         * the QR preconditioning, else BBP_EGEOM) */
  int32_t precision;    /* bbp_precision */
  int32_t trunc;        /* bbp_trunc */
  int32_t rsvd_q;       /* T2 power iterations */
  int32_t rsvd_p;       /* T2 oversampling */
  uint64_t seed;        /* T2 sketch seed */
  void* stream;         /* borrowed hipStream_t; NULL: the library creates one */
  int64_t hbm_budget_bytes; /* > 0: device memory the handle may take (resident
                             * state plus workspace); create fails with
                             * BBP_ENOMEM before allocating anything when the
                             * plans need more.  0: no limit */
  int32_t swallow_order;    /* order of the sums in a swallow (the same value):
                             * 0 the cheaper by the plan's cost model, 1 merge
                             * the in-leg run first, 2 absorb the ket tensor
                             * site by site along the run */
  int32_t hermitize;        /* 1: every new message A is replaced by
                             * (A + A^dagger) / 2, A^dagger exchanging the ket
                             * and bra index of each double leg and
                             * conjugating (Sec. "'Hermitize' MPSs"); 0: off */
  double damping;           /* 1 - alpha of the learning step (Eq.
                             * blockBP:kagome:numerics:learning_step1): the
                             * stored message becomes (1 - damping) new +
                             * damping old; in [0, 1), 0: the new message
                             * alone.  With hermitize or damping on, each MPS
                             * sum is brought to right-canonical form with
                             * unit norm and compressed to chi by exact SVDs,
                             * so chi must be at most 72 (bonds of the sum up
                             * to 2 chi), else BBP_EINVAL */
} pepsnet_desc;

/* Build the problem the thesis states for BlockBP (the lattice, its blocks
 * and their faces; Sec. "Defining the Kagome block" for the hexagonal block
 * of the infinite lattice, Eq. blockBP:DefiningEquation for the finite
 * patch; free parameters d, D, chi and the block size, Ch. "ITE for Kagome
 * using BlockBP"), compile the static plans of the message updates and
 * expectations, allocate device memory and copy the site tensors (host
 * pointer, complex128, see tensor order above; `sites_len` in doubles) to
 * the device.  Messages start as vec(I_D)/sqrt(D) on every leg (a positive
 * semi-definite start).  Inputs are copied; *out receives the handle, which
 * owns all of its device memory.  Errors: BBP_EINVAL (bad descriptor or
 * site buffer length; nothing allocated), BBP_EGEOM (the block or sweep
 * order cannot be built), BBP_ENOMEM (over the HBM budget or allocation
 * failure), BBP_EDEVICE, BBP_ENUMERIC (non-finite site tensor entry). */
int32_t pepsnet_create(const pepsnet_desc* desc, const double* sites, int64_t sites_len,
                       pepsnet_t* out);

/* Replace the site tensors (same shapes); messages are kept (warm start)
 * unless reset_messages != 0. */
int32_t pepsnet_set_sites(pepsnet_t h, const double* sites, int64_t sites_len,
                          int32_t reset_messages);

/* Run BlockBP sweeps (Alg. BlockBP_singleBlock on the infinite lattice: the
 * message computed toward a face replaces the message on the opposite face;
 * Eq. blockBP:DefiningEquation on a finite patch).  Each message is the
 * contraction of its block with the other incoming messages by the
 * boundary-MPS method, compressed to bond chi (Sec. "The boundary-MPS
 * method"); every message of a sweep is computed from the previous sweep's
 * messages (Jacobi).  Stops after max_sweeps or when the largest Frobenius
 * distance between a message and its previous value (both unit norm, real
 * positive trace; Eq. bp:convergenceCriterium) is <= tol.  *sweeps_done and
 * *max_err (may be NULL) receive the sweeps run and the last distance.
 * Returns BBP_OK, BBP_NOT_CONVERGED (tol not reached; outputs valid),
 * BBP_EINVAL (max_sweeps < 0, workspace released), BBP_ENUMERIC (a message
 * became non-finite; the sweep that produced it is counted) or
 * BBP_EDEVICE. */
int32_t blockbp_sweep(pepsnet_t h, int32_t max_sweeps, double tol, int32_t* sweeps_done,
                      double* max_err);

/* For callers that cannot allocate device memory (serving loops and
 * harnesses that forbid hipMalloc): blockbp_sweep without any allocation.
 * The sweep's workspace and launch descriptors live in a fixed device array
 * of the library, PEPSNET_NOALLOC_MAX_BYTES (128 MiB) on each device it runs
 * on, held until the process ends, instead of in the handle's workspace
 * (which may be released).  Arguments, results and messages as for
 * blockbp_sweep; launches are direct (no graph).  BBP_ENOMEM if the handle's
 * workspace (pepsnet_memory) plus its descriptors exceed the array;
 * BBP_EDEVICE if the array's address could not be resolved when the handle
 * was created.  Every call on a device shares that device's array and
 * rewrites it (descriptors uploaded, workspace cleared) on entry: calls that
 * overlap in time on one device race, from any stream or thread. */
#define PEPSNET_NOALLOC_MAX_BYTES (128LL << 20)
int32_t blockbp_sweep_noalloc(pepsnet_t h, int32_t max_sweeps, double tol, int32_t* sweeps_done,
                              double* max_err);

/* Local expectation values from the current messages: for every requested
 * bond (i, j) the two-site reduced density matrix rho_ij is contracted from
 * the block holding the bond with sites i and j left open and every incoming
 * message absorbed (on a finite patch, the one or two blocks holding i and
 * j), and <O> = Tr(rho_ij O) / Tr(rho_ij) for each requested operator.  The
 * default operator is the Heisenberg bond term S_i . S_j with S = sigma / 2
 * (Eq. res:afm-h:hamiltonian).
 *   bond_ids: n_bonds indices into the bond table of pepsnet_bonds (the six
 *             unique bonds of the central unit cell of the infinite lattice:
 *             U-DL, U-DR, DL-DR, DR-DL(a1), U-DL(a2), U-DR(a2-a1); every
 *             bond of a finite patch, ordered by first site then slot);
 *             distinct; NULL: the whole table (n_bonds ignored).
 *   ops:      n_ops operators, each 4 x 4 complex, row-major, in the basis
 *             (p_i p_j) with p_i the bond's first site: ops[k][r][c] =
 *             <r| O_k |c> (r, c = p_i * 2 + p_j); n_ops <= 64.  NULL: one
 *             operator, S_i . S_j (n_ops ignored).
 *   out:      n_bonds x n_ops complex <O_k> (NULL to skip).
 *   rho_out:  n_bonds x 4 x 4 complex rho_ij, row (p_i p_j), column
 *             (p_i' p_j'), not normalised (NULL to skip).
 *   energy:   energy per site, (1/3) sum of <S . S> over the six unique bonds
 *             (infinite lattice) or the mean bond energy (finite patch); only
 *             with bond_ids NULL (else it must be NULL).
 *   n_bonds_out: the number of bonds evaluated (may be NULL).
 * Returns BBP_OK, BBP_EINVAL (bad ids or counts, energy with a bond subset,
 * workspace released), BBP_ENUMERIC (zero or non-finite trace) or
 * BBP_EDEVICE.  The first call with a new bond subset compiles its plan and
 * allocates its descriptors. */
int32_t blockbp_expect(pepsnet_t h, int32_t n_bonds, const int32_t* bond_ids, int32_t n_ops,
                       const double* ops, double* out, double* rho_out, double* energy,
                       int32_t* n_bonds_out);

/* Two-site measures of the density matrices the last blockbp_expect call
 * computed: the negativity of rho_ij with the partial transpose on the second
 * site (Eq. res:negativity) and, when sigma is given, the fidelity
 * F(rho_ij, sigma_k) (Eq. metrics:fidelity).  Both matrices are normalised to
 * unit trace and taken Hermitian; eigenvalues below zero (rounding) count as
 * zero under the square roots, so F loses accuracy like sqrt(eps) when a
 * matrix is rank-deficient.  bond_ids: n_bonds ids of the default bond table
 * (NULL: all, n_bonds = their number); every listed bond's rho must come
 * from a blockbp_expect call made since the last sweep or site/message
 * replacement, else BBP_EINVAL.  sigma: NULL or n_bonds 4x4 complex matrices,
 * row-major in the (p_i p_j) basis; negativity / fidelity: n_bonds doubles
 * each (may be NULL; fidelity needs sigma).  Computed on the device. */
int32_t blockbp_rho_measures(pepsnet_t h, int32_t n_bonds, const int32_t* bond_ids,
                             const double* sigma, double* negativity, double* fidelity);

/* Number of bonds in the bond table and their site pairs (2 ints per bond). */
int32_t pepsnet_bonds(pepsnet_t h, int32_t* pairs, int32_t cap, int32_t* n);

/* Copy the current messages to host (complex128, each message's sites in
 * order, every site zero-padded to its static shape).  With buf NULL only
 * *len (doubles) is set. */
int32_t pepsnet_get_messages(pepsnet_t h, double* buf, int64_t cap, int64_t* len);
int32_t pepsnet_set_messages(pepsnet_t h, const double* buf, int64_t len);

/* Static shape of message slot m site j: (bond left, double-leg dim, bond right). */
int32_t pepsnet_message_shape(pepsnet_t h, int32_t m, int32_t j, int32_t* l, int32_t* P,
                              int32_t* r, int32_t* n_sites);
int32_t pepsnet_num_messages(pepsnet_t h);

/* Stream that the handle launches on (hipStream_t). */
void* pepsnet_stream(pepsnet_t h);

/* Time the last sweep's kernels with HIP events on the handle's stream:
 * average milliseconds per sweep over the sweeps run since the last reset. */
int32_t pepsnet_timing(pepsnet_t h, int32_t reset, double* ms_per_sweep, int64_t* sweeps);

/* Use a captured HIP graph for sweeps (1) or direct launches (0). */
int32_t pepsnet_use_graph(pepsnet_t h, int32_t on);

/* Streams a sweep may use, 1 to 4 (default 4).  The message updates of a
 * sweep are independent (Sec. "The Block Belief-Propagation Algorithm":
 * every update reads only the previous sweep's messages), so updates whose
 * kernel sequences differ run on separate streams, forked from and joined
 * back into the handle's stream; 1 issues every launch on the handle's
 * stream.  Results are bit-identical either way.  BBP_EINVAL outside
 * [1, 4]. */
int32_t pepsnet_use_streams(pepsnet_t h, int32_t n);

/* Algorithmic flop count of one sweep's contraction GEMMs (8 real flops per
 * complex multiply-add) and of all its GEMMs, and the number of launches. */
int32_t pepsnet_sweep_stats(pepsnet_t h, double* contraction_flops, double* gemm_flops,
                            int64_t* launches);

/* Per-kernel live timing: run n_sweeps sweeps with HIP events recorded on
 * the handle's stream around every launch and accumulate, per kernel slot
 * (slot = kind * 3 + precision for GEMMs, kind * 3 otherwise, kinds: 0 GEMM,
 * 1 transpose, 2 QR, 3 truncated SVD, 4 sketch, 5 norm, 6 pad, 7 message
 * phase, 8 split gauge, 9 Cholesky step of the tall QR, 10 sum of split-K
 * partial products; slot 7 is the
 * blocked QR for working copies that overflow LDS; the truncated SVD is
 * slot 9 through one-sided Jacobi, or slot 10 for its bidiagonalisation
 * kernel and slot 11 for the kernel computing the kept values and vectors),
 * the elapsed milliseconds, the launch count, and the algorithmic flops (8
 * per complex multiply-add) and bytes of the launches.  The Gram and Q
 * products of the tall QR count as GEMMs.  Arrays hold
 * PEPSNET_PROFILE_SLOTS entries; NULL skips an output. */
#define PEPSNET_PROFILE_SLOTS 33
int32_t pepsnet_profile_sweeps(pepsnet_t h, int32_t n_sweeps, double* ms, int64_t* launches,
                               double* flops, double* bytes);

/* Run one sweep launch by launch with a HIP event after each launch and
 * report, per launch of the sweep's launch list, 10 doubles: op kind (as
 * above), precision, kernel variant, items, largest M, N, K (GEMM) or rows,
 * cols (factorisations), algorithmic flops, algorithmic bytes, milliseconds.
 * With rec NULL only *n (launches) is set; cap counts doubles. */
int32_t pepsnet_profile_launches(pepsnet_t h, double* rec, int64_t cap, int64_t* n);

/* ---- batched sweeps (independent blocks of uneven N, D, chi in one launch
 * sequence).  BlockBP message updates of different blocks are independent
 * (Sec. "The Block Belief-Propagation Algorithm", complexity discussion:
 * the sides can be computed in parallel); a batch merges the sweep plans of
 * n handles so that every kernel launch serves the same stage of every
 * handle's message updates, optionally replayed as one captured HIP graph.
 * Results are bit-identical to sweeping each handle on its own. */
typedef struct pepsnet_batch_s* pepsnet_batch_t;

/* Merge the sweep plans of hs[0..n) (distinct handles, borrowed: they must
 * outlive the batch).  stream: borrowed hipStream_t, NULL to create one. */
int32_t pepsnet_batch_create(const pepsnet_t* hs, int32_t n, void* stream, pepsnet_batch_t* out);
int32_t pepsnet_batch_use_graph(pepsnet_batch_t b, int32_t on);
/* Run `sweeps` Jacobi sweeps of every handle.  max_err[i] (n doubles, may be
 * NULL) receives handle i's largest message distance of the last sweep, *ms
 * (may be NULL) the device time of the sweeps from HIP events.  Fails with
 * BBP_EINVAL if a handle was swept on its own since the batch was made. */
int32_t blockbp_sweep_batch(pepsnet_batch_t b, int32_t sweeps, double* max_err, double* ms);
/* GEMM flops of one merged sweep and its number of kernel launches. */
int32_t pepsnet_batch_stats(pepsnet_batch_t b, double* gemm_flops, int64_t* launches);
void pepsnet_batch_destroy(pepsnet_batch_t b);

/* ---- device memory of a handle.  Resident: site tensors, their permuted
 * matrices, both message sets, expectation outputs and descriptors.
 * Workspace: the boundary chains and scratch of the message updates, needed
 * only while a sweep or expectation runs.  Releasing it keeps the state
 * (messages stay on the device); acquiring it again re-resolves the launch
 * descriptors (batches made before become invalid).  Sweeps, expectations
 * and profiling fail with BBP_EINVAL while the workspace is released. */
int32_t pepsnet_memory(pepsnet_t h, int64_t* resident_bytes, int64_t* workspace_bytes);
int32_t pepsnet_release_workspace(pepsnet_t h);
int32_t pepsnet_acquire_workspace(pepsnet_t h);

/* GEMM tile autotuner.  Times every tile shape of k_gemm (64x64, 16x64,
 * 64x16, 64x80, 80x64) on one launch of each distinct GEMM shape (precision,
 * M, N, K, operand ops, scattered store) of the handle's sweep plans, with
 * the outputs redirected to a temporary buffer so the handle's state is not
 * touched, keeps the fastest per shape and recompiles the plans with it
 * (batches made afterwards use it too).  Results are bit-identical to the
 * untuned plans: the tile shape never changes the order of any element's
 * sum.  cache_path (NULL: none) is a text file of earlier choices, one line
 * per shape; shapes found there are not timed, and the file is rewritten
 * with the union.  *n_timed / *n_shapes (may be NULL) get the shapes timed
 * now and the shapes tuned in all.  Needs the workspace (BBP_EINVAL when
 * released); allocates a temporary output buffer for the timing. */
int32_t pepsnet_autotune(pepsnet_t h, const char* cache_path, int32_t* n_timed, int32_t* n_shapes);

/* ---- serving loop (continuous batching of expectation requests on
 * resident states).  A request on a state optionally replaces its site
 * tensors (an imaginary-time step: messages are kept, a warm start as in the
 * thesis's ITE algorithm), sweeps to tol or max_sweeps and evaluates the
 * default bonds' <S_i . S_j> and the energy per site.  A worker thread admits
 * queued requests in arrival order whenever an in-flight slot is free and a
 * workspace slot fits (a request that does not fit lets later ones pass; one
 * request per state at a time) and advances every in-flight request on its
 * state's own stream, so requests overlap on the device.  A state whose
 * workspace is released borrows a server workspace slot for the request's
 * duration; the server allocates at most max_inflight slots within
 * hbm_budget_bytes as its pool grows and keeps them until it is destroyed,
 * and a state that gets back the slot it held last keeps its resolved launch
 * descriptors, so steady-state admission and completion allocate and free no
 * device memory (slots are freed only to fit a larger state).  Results are
 * those of running the request alone.  States must not be used by the caller
 * while they have requests in the server; give each state its own stream
 * (desc stream NULL) for overlap.  submit and poll are thread-safe. */
typedef struct bbp_server_s* bbp_server_t;
int32_t bbp_server_create(int64_t hbm_budget_bytes, int32_t max_inflight, bbp_server_t* out);
/* new_sites: NULL (unchanged) or sites_len doubles as for pepsnet_set_sites. */
int32_t bbp_server_submit(bbp_server_t s, pepsnet_t state, const double* new_sites,
                          int64_t sites_len, double tol, int32_t max_sweeps, uint64_t* ticket);
/* Collect a request: BBP_PENDING if not finished and wait == 0; otherwise the
 * request's code (BBP_OK, BBP_NOT_CONVERGED or an error) with the outputs:
 * energy per site, up to cap bond values (*n_bonds gets the count), sweeps
 * run, last message distance, the submit-to-completion latency in seconds
 * and gpu_window_ms[2], the device-side start and end of the request's work
 * in ms since the server was created (from events on the state's stream; NaN
 * if the request failed early).  Every output pointer may be NULL.  A ticket
 * is collected once. */
int32_t bbp_server_poll(bbp_server_t s, uint64_t ticket, int32_t wait, double* energy_per_site,
                        double* bond_ss, int32_t cap, int32_t* n_bonds, int32_t* sweeps_done,
                        double* max_err, double* latency_s, double* gpu_window_ms);
/* Peak bytes of workspace slots held and peak in-flight requests so far,
 * requests completed, requests still queued, and the number of workspace
 * slot allocations made (it stops growing once the pool is warm). */
int32_t bbp_server_stats(bbp_server_t s, int64_t* peak_bytes, int32_t* peak_inflight,
                         int64_t* completed, int32_t* queued, int64_t* slot_allocations);
/* Finishes queued and in-flight requests, then stops the worker. */
void bbp_server_destroy(bbp_server_t s);

void pepsnet_destroy(pepsnet_t h);
const char* pepsnet_last_error(void);

/* Host-only geometry queries (no device use), for checking the sweep orders
 * against an independent implementation.
 *   what = 0: faces of block `a`: [n_faces, {keytype, key, n_legs, (site, slot)...}...]
 *   what = 1: sweep of block `a` toward face `b` with open sites:
 *             [n_steps, {site, pos, r, s, in_slots[r], out_slots[s], open, absorb}...,
 *              n_final, (site, slot)...]
 *   what = 2: summary [n_sites, n_blocks, n_msgs, n_bonds]
 * buf receives up to cap int32 values; *len gets the needed length. */
int32_t pepsnet_describe(const pepsnet_desc* desc, int32_t what, int32_t a, int32_t b,
                         int32_t n_open, const int32_t* open_sites, int32_t* buf, int64_t cap,
                         int64_t* len);

#ifdef __cplusplus
}
#endif

#endif /* PEPSNET_H */
