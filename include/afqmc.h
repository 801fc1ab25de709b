/*
 * afqmc.h - C ABI of the MI355X (gfx950) correlated-sampling phaseless AFQMC
 * walker step (Shee, Zhang, Reichman, Friesner; arXiv:1703.01545).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All matrices are row-major float64 unless stated otherwise.
 * - Host input arrays are borrowed for the duration of the call and copied;
 *   the library never keeps or frees caller memory.
 * - Handles own their device memory (allocated with hipMalloc in
 *   afqmc_load_hamiltonian / afqmc_init_walkers) until afqmc_free_*.
 * - Work is enqueued on the HIP stream given to afqmc_load_hamiltonian
 *   (NULL = the null stream).  Calls that return host data synchronise that
 *   stream before returning.
 * - Every call returns an afqmc_status; on failure a message is available
 *   from afqmc_last_error() (thread-local).  No call aborts, exits or throws
 *   across the ABI.
 * - Handles are not synchronised internally: calls on one handle, or on
 *   systems that share a Hamiltonian (and so its stream), must not overlap.
 *   Calls on unrelated Hamiltonians may come from different host threads;
 *   the process-wide caches (tuned launch shapes, captured batch graphs)
 *   are guarded.
 * - A walker whose weight is no longer positive is frozen, not an error
 *   (Sec. II.B of the paper); afqmc_get_walkers reports it through `alive`.
 */
#ifndef AFQMC_H
#define AFQMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AFQMC_OK = 0,
    AFQMC_E_INVALID = -1,  /* null pointer, bad enum, non-positive size     */
    AFQMC_E_SHAPE = -2,    /* inconsistent sizes, or a pair that does not
                              share M, n_chol, walker count and L (Sec. II.C) */
    AFQMC_E_NOMEM = -3,    /* device allocation failed                      */
    AFQMC_E_DEVICE = -4,   /* a HIP runtime call or kernel launch failed    */
    AFQMC_E_SINGULAR = -5, /* initial determinant orthogonal to the trial   */
    AFQMC_E_STATE = -6     /* call out of order (e.g. pair at different t)  */
} afqmc_status;

/* Arithmetic of the Cholesky contractions (force bias, field sum, exchange)
 * and of the propagator products.
 * AFQMC_FP64: everything in FP64 (the parity path).
 * AFQMC_FP32: L, L^half, Theta and the field coefficients held in FP32, FP32
 *   MFMA with FP32 accumulation; propagator products in FP32.
 * AFQMC_BF16: the Cholesky contractions on the BF16 matrix cores with split
 *   operands (each FP32 operand carried as hi + lo BF16, three products per
 *   pair, FP32 accumulation; relative error a few 2^-17); propagator
 *   products (one-body halves and Taylor terms) in FP32.
 * AFQMC_BF16_PLAIN: L, L^half, Theta and the field coefficients stored as
 *   single BF16 values, one BF16 product per pair (fastest, least accurate).
 * AFQMC_BF16X3: as AFQMC_BF16, and the propagator products also in split
 *   BF16: the Taylor terms (A_w carried as hi + lo planes) and the one-body
 *   halves, applied as P y = y + Q y with Q = P - I (formed in FP64, carried
 *   as hi + lo planes) so that the identity part is added exactly in FP32
 *   and the rounding of the product scales with |Q|.  Any M: the operand
 *   tiles are zero-padded to 16 rows and 32 columns.
 * In every mode the walker determinants, overlaps, determinants,
 * Gram-Schmidt, weights and phases stay FP64. */
typedef enum {
    AFQMC_FP64 = 0,
    AFQMC_FP32 = 1,
    AFQMC_BF16 = 2,
    AFQMC_BF16_PLAIN = 3,
    AFQMC_BF16X3 = 4
} afqmc_prec;

/* Projection variant.  PHASELESS: the ph-AFQMC step of Sec. II.A with the
 * hybrid weight of Sec. II.D.  FREE: free projection (no force bias, complex
 * weight, no phase projection), Sec. II.A. */
typedef enum { AFQMC_PHASELESS = 0, AFQMC_FREE = 1 } afqmc_mode;

typedef struct afqmc_ham_s* afqmc_ham; /* Hamiltonian: h, L, e_core        */
typedef struct afqmc_sys_s* afqmc_sys; /* one system: ham + trial + walkers */

typedef struct {
    double dt;            /* imaginary time step (Eq. 3)                    */
    int taylor_order;     /* order K of the Taylor series for the HS factor */
    int ortho_every;      /* modified Gram-Schmidt period in steps (0: off) */
    int measure_every;    /* mixed-energy period in steps (0: off)          */
    afqmc_prec contract_prec;
    afqmc_mode mode;
    /* Optional force-bias cap, one of the bounding conditions Sec. II.D
     * cites without stating.  fb_cap > 0: every step counts the (live
     * walker, gamma) with |xbar_gamma| > fb_cap (afqmc_cap_events); with
     * caps_enabled those xbar_gamma are also scaled to modulus fb_cap, phase
     * kept.  fb_cap = 0 (the default): no cap, nothing counted. */
    double fb_cap;
    int caps_enabled;
} afqmc_params;

/* Load H of Eq. 1: h1 (M x M, symmetric), chol (n_chol x M x M, each
 * L^gamma symmetric, V_ijkl = sum_gamma L^gamma_ik L^gamma_jl), e_core.
 * hip_stream: hipStream_t (or NULL) on which all later work of systems built
 * on this Hamiltonian is enqueued.  Errors: E_INVALID (null/size <= 0),
 * E_NOMEM, E_DEVICE. */
afqmc_status afqmc_load_hamiltonian(int M, int n_chol, const double* h1, const double* chol,
                                    double e_core, void* hip_stream, afqmc_ham* out);

/* Build one system on `ham`: trial determinant (M x (n_alpha + n_beta),
 * column j = orbital j, alpha columns first; real, Sec. II.A) and n_walkers
 * walkers initialised to init_phi (same shape; NULL -> the trial; a
 * different determinant such as ROHF walkers with a UHF trial, Sec. II.D),
 * weight 1.  Precomputes the mean-field shift a_gamma = Tr(L_gamma G_T)
 * (Eq. 2, 9), the one-body exponential P = exp(-dt h~/2) with
 * h~ = h - 1/2 sum L_g L_g + sum a_g L_g, and the half-rotated L^half, h^half.
 * Errors: E_INVALID, E_SHAPE (n_alpha/n_beta outside [0, M] or both 0),
 * E_SINGULAR (init overlap with the trial is zero), E_NOMEM, E_DEVICE. */
afqmc_status afqmc_init_walkers(afqmc_ham ham, int n_alpha, int n_beta, const double* trial,
                                const double* init_phi, int n_walkers, const afqmc_params* params,
                                afqmc_sys* out);

/* As afqmc_init_walkers with a multi-determinant trial (Sec. II.D, the
 * CASSCF trial): phi_T = sum_i coeffs[i] D_i, dets: n_det determinants of
 * shape M x (n_alpha + n_beta) (row-major, column j = orbital j, alpha
 * first), coeffs: n_det real coefficients; walkers start from init_phi or
 * from D_0.  The overlap <phi_T|phi> = sum_i c_i <D_i|phi>, the force bias
 * and the mixed local energy are the r_i = c_i <D_i|phi> / <phi_T|phi>
 * weighted sums of those against each D_i; the mean-field shift is
 * a_g = <phi_T|rho_g|phi_T> / <phi_T|phi_T> of the whole expansion.  Cost
 * and memory of the overlaps, force bias and energy grow linearly with
 * n_det; the propagation is unchanged.  n_det = 1 is afqmc_init_walkers.
 * Errors: as afqmc_init_walkers; E_INVALID (n_det outside 1..256, null
 * coefficients); E_SINGULAR also when two determinants have exactly
 * orthogonal spin blocks (the pair term of a_g is then not formed from
 * their overlap) or the expansion has zero norm.  The reverse-mode adjoint
 * refuses such systems (E_STATE). */
afqmc_status afqmc_init_walkers_msd(afqmc_ham ham, int n_alpha, int n_beta, int n_det,
                                    const double* coeffs, const double* dets,
                                    const double* init_phi, int n_walkers,
                                    const afqmc_params* params, afqmc_sys* out);

/* Advance every live walker n_steps imaginary-time steps (force bias Eq. 8-9,
 * propagator Eq. 11 by Taylor series between one-body halves, overlap ratio
 * and phaseless hybrid weight, Sec. II.A/II.D; modified Gram-Schmidt every
 * ortho_every steps, Sec. II.D).  Fields: `fields` NULL -> counter-based
 * Philox4x32-10 normals keyed by (seed, stream_id, absolute step t, walker k,
 * gamma); else a DEVICE pointer to n_steps x n_walkers x n_chol float64
 * values (C order), read for steps t0 .. t0+n_steps-1.  Measurements are not
 * taken here (see afqmc_local_energy / afqmc_pair_step).
 * Errors: E_INVALID, E_STATE (freed handle), E_DEVICE. */
afqmc_status afqmc_step(afqmc_sys sys, uint64_t seed, uint64_t stream_id, int n_steps,
                        const double* fields);

/* Mixed local energy of every walker, Eq. 7 and Eq. 10:
 * E_L = e_core + sum_s Tr(h^half_s Theta^s)
 *       + 1/2 sum_g [(sum_s Tr T_gs)^2 - sum_s Tr(T_gs T_gs)],
 * T_gs = L^half_gs Theta^s, and the phaseless mixed estimator
 * e_mixed = sum_k w_k Re E_L,k / sum_k w_k over live walkers (free mode:
 * Re(sum W E_L / sum W)).  e_local: host, n_walkers x 2 (re, im) or NULL;
 * weights: host, n_walkers (free mode: n_walkers x 2) or NULL; e_mixed: host,
 * 1 double, or NULL.  Synchronises.  Errors: E_INVALID, E_DEVICE. */
afqmc_status afqmc_local_energy(afqmc_sys sys, double* e_local, double* weights, double* e_mixed);

/* Modified Gram-Schmidt of each spin block of every live walker (Sec. II.D);
 * overlaps and Theta are recomputed, weights unchanged (Eq. 6). */
afqmc_status afqmc_orthonormalize(afqmc_sys sys);

/* Correlated pair (Sec. II.B): advance a and b n_steps with identical fields
 * (walker k of a and of b draw the same x at every step and gamma), no
 * population control, MGS every ortho_every steps, and every measure_every
 * steps record E_a, E_b and dE = E_b - E_a.  e_trace: host array of
 * (n_steps / measure_every) x 3 doubles, or NULL.  `fields` as in afqmc_step
 * (one device array shared by both systems).  Errors: E_SHAPE when the two
 * systems differ in M, n_chol, walker count or L (Sec. II.C), or in
 * dt/ortho_every/measure_every; E_STATE when their step counters differ. */
afqmc_status afqmc_pair_step(afqmc_sys a, afqmc_sys b, uint64_t seed, int n_steps,
                             const double* fields, double* e_trace);

/* Number of (live walker, step, gamma) whose force bias exceeded fb_cap
 * since the system was created (counted whether or not the cap is applied;
 * always 0 with fb_cap = 0).  Synchronises. */
afqmc_status afqmc_cap_events(afqmc_sys sys, int64_t* count);

/* Gram-Schmidt monitor (Sec. II.D: the walker orbitals lose orthogonality
 * between orthonormalisations).  Every orthonormalisation of a live walker's
 * spin block records ell = max_k 1/2 ln(S_kk / D_k), with S = Phi^H Phi =
 * L D L^H over the block's columns (0 for orthogonal columns; about
 * 2 ell / ln 10 decimal digits of the Gram-matrix factorisation are lost),
 * and |ln |det R|| = |1/2 sum_k ln D_k| (how far the columns' volume moved
 * since the previous orthonormalisation); non-finite values count as
 * infinite.  Returns (each pointer may be NULL) the largest ell and the
 * largest |ln |det R|| over the walker spin blocks since the system was
 * created or the last call, and how many blocks had ell > threshold at some
 * orthonormalisation; then clears the record.  Errors: E_INVALID (threshold
 * negative or NaN), E_STATE.  Synchronises. */
afqmc_status afqmc_gs_monitor(afqmc_sys sys, double threshold, double* max_ell,
                              double* max_lndet, int64_t* trips);

/* Population control by the comb (Sec. II.B: walkers with large weights are
 * replicated, small ones stochastically removed), for the equilibration of a
 * primary system; not used between correlated systems.  With C the running
 * sum of the live weights in walker order and W its last value, new walker j
 * copies the first walker k with C[k] > (j + xi) W / n_walkers; every new
 * walker is live with weight W / n_walkers (the total weight is kept).  xi:
 * one uniform number in [0, 1), drawn by the caller.  Overlaps and Theta are
 * recomputed for the copies.  Synchronises.  Errors: E_INVALID (xi outside
 * [0, 1)), E_STATE (free mode, or no walker of positive weight: nothing
 * changed). */
afqmc_status afqmc_population_control(afqmc_sys sys, double xi);

/* Preliminary equilibration scheme (Sec. II.B): start the secondary system
 * from the primary's walkers.  Walker k of `sec` takes walker k's
 * determinant of `pri` (the first n_alpha and n_beta orbital columns of each
 * spin block when the secondary has fewer electrons), and its weight becomes
 * w_pri |r| max(0, cos arg r) with r = <phi_T^sec|phi> / <phi_T^pri|phi> (the
 * phase of the ratio projected as in the phaseless step; a walker with
 * cos arg r <= 0 is frozen).  The secondary's step counter is set to the
 * primary's, so the two continue as a correlated pair.  Synchronises.
 * Errors: E_SHAPE (different M or walker count, more electrons of a spin
 * in the secondary, different streams), E_STATE (free mode), E_INVALID. */
afqmc_status afqmc_init_from_primary(afqmc_sys sec, afqmc_sys pri);

/* For callers that cannot allocate device memory during the call (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): afqmc_pair_step with the same arguments, results and errors,
 * bit for bit, except that the device staging rows of the energy trace live
 * in a fixed array inside the library (one per GPU, held until the process
 * ends) instead of a buffer allocated per call; the call itself makes no
 * hipMalloc or hipFree.  At most AFQMC_NOALLOC_MAX_MEASUREMENTS measurement
 * steps per call (else E_INVALID, nothing run); profiling must be off
 * (E_STATE: it creates events).  Every call on one GPU shares that array:
 * calls that overlap on one GPU (different host threads or streams) race on
 * it.  Each row is written before it is read, so nothing needs clearing
 * between calls.  The systems themselves are allocated beforehand by
 * afqmc_init_walkers. */
#define AFQMC_NOALLOC_MAX_MEASUREMENTS 1024
afqmc_status afqmc_pair_step_noalloc(afqmc_sys a, afqmc_sys b, uint64_t seed, int n_steps,
                                     const double* fields, double* e_trace);

/* Many correlated pairs of uneven size advanced together (the pairs of
 * Sec. II.B, batched).  Pair p (systems a[p], b[p]) runs exactly what
 * afqmc_pair_step(a[p], b[p], seeds[p], n_steps, NULL, ...) runs, bit for
 * bit.  The pairs are spread over `lanes` streams (largest first onto the
 * least-loaded lane; lanes <= 0 picks 4).  One period of
 * lcm(ortho_every, measure_every) steps (doubled when odd) of every pair is
 * captured once into a HIP graph with fork/join edges between the lanes and
 * replayed for each whole period; the Philox step word and the trace slot
 * are read from device counters, so one graph serves every period.  Steps
 * before the first period boundary and after the last one are launched
 * directly.  Every system is autotuned (afqmc_autotune) before capture.
 * Graphs are cached per (handles, seeds, lanes) until a handle is freed.
 * flags bit 0: no graph, launch every step directly (same lanes).
 * e_traces: host, n_pairs x n_meas x 3 doubles (E_a, E_b, dE), n_meas =
 * number of measurement steps among the n_steps, or NULL.  Errors: as
 * afqmc_pair_step for each pair; E_STATE when the systems are not all at
 * the same step; E_SHAPE when they differ in dt, periods or mode, or do not
 * share one stream; E_INVALID for null arrays or a handle used twice.
 * Synchronises. */
afqmc_status afqmc_pair_batch_step(int n_pairs, const afqmc_sys* a, const afqmc_sys* b,
                                   const uint64_t* seeds, int n_steps, int lanes, int flags,
                                   double* e_traces);

/* Reverse-mode derivative of the mixed energy (Eq. 7, Eq. 10) with respect to
 * a one-body perturbation h -> h + lambda V, at lambda = 0 (the system's own
 * h).  The paper has no derivative; its correlated pairs at +-lambda are the
 * finite differences this is checked against.
 * afqmc_adjoint_forward advances the system n_steps exactly as afqmc_step
 * with device fields (seed, stream id 0) would, keeping a snapshot of the
 * walkers every checkpoint_every steps, and returns the mixed energy after the
 * last step (measured there whatever measure_every says).  lambda enters the
 * one-body halves P of every step of this window and h^half of the final
 * local energy; the fields are held fixed (pathwise derivative).
 * afqmc_adjoint_backward recomputes the window one segment at a time from
 * the snapshots and returns dE/dlambda; the system is left in the state after
 * the window.  With checkpoint_every >= n_steps (one segment) the forward
 * pass records every step instead (device memory of about
 * n_steps (1 + 1/ortho_every) walker blocks of nw 2 N M doubles) and the
 * backward pass recomputes nothing; the result is bitwise the same.  Steps
 * whose propagation runs FP64 or FP32 products also record their Taylor
 * terms (taylor_order + 1 more walker blocks per step) when these fit in 3/4
 * of the free device memory, and the reverse pass starts from them.  Systems
 * with an applied force-bias cap or a multi-determinant trial are refused
 * (E_STATE): the reverse pass differentiates the uncapped single-determinant
 * step.  V: host M x M symmetric, row-major, copied.  prec: AFQMC_FP64
 * or AFQMC_FP32 products in the adjoint's contractions (FP64 storage and
 * small dense algebra).  Errors: E_STATE (free mode; backward without a
 * forward), E_SHAPE (a spin block above 64 orbitals), E_INVALID.
 * Synchronises. */
afqmc_status afqmc_adjoint_forward(afqmc_sys sys, const double* V, uint64_t seed, int n_steps,
                                   int checkpoint_every, afqmc_prec prec, double* energy);
afqmc_status afqmc_adjoint_backward(afqmc_sys sys, double* dE_dlambda);

/* Launch-shape autotuner.  Times every candidate launch shape of the
 * force-bias and field-sum GEMMs (64 x 64, 128 x 128 or 256 x 128 tiles, the last
 * over 8 or, for split BF16, 16 wavefronts) and of the
 * fused propagation (waves per workgroup x column blocks per wave, B
 * prefetch or not, orbitals per workgroup) on this system's own buffers and keeps the fastest per
 * problem shape in a process-wide table, so tuning another system of the
 * same shape costs nothing.  All candidates sum in the same order, so tuning
 * never changes a result bit.  The walker state is left unchanged.  choice
 * (optional, host, 3 ints): the chosen force-bias tile and field-sum tile
 * (1: 64 x 64, 2: 128 x 128, 3: 256 x 128, 4: 256 x 128 over 16 wavefronts)
 * and the propagation shape index.
 * Synchronises. */
afqmc_status afqmc_autotune(afqmc_sys sys, int* choice);

/* The autotuner's table on disk, so that a new process need not time the
 * candidates again.  afqmc_tune_cache_save writes every problem shape tuned
 * in this process with its choice, tagged with the current device's
 * architecture and compute-unit count and a format version.
 * afqmc_tune_cache_load reads such a file, checks the version and that it
 * was written on a device like the current one, checks every entry (a
 * choice the tuner could have made for its shape), and only then adds the
 * entries; shapes already tuned in this process keep their choice.  Any
 * failed check leaves the table as it was.  Errors: E_INVALID (NULL or
 * unreadable / unwritable path, another version, another device, a
 * malformed entry), E_DEVICE (no current device).  afqmc_tune_cache_clear
 * empties the table (systems keep the shapes already chosen for them; the
 * next afqmc_autotune of a shape times its candidates again). */
afqmc_status afqmc_tune_cache_save(const char* path);
afqmc_status afqmc_tune_cache_load(const char* path);
afqmc_status afqmc_tune_cache_clear(void);

/* Read back walker state: phi (n_walkers x 2 x N x M: plane 0 = real,
 * plane 1 = imaginary part of orbital column i, N = n_alpha + n_beta),
 * w (n_walkers; free mode n_walkers x 2), log_ovlp (n_walkers x 2:
 * ln <phi_T|phi>, imaginary part modulo 2 pi), alive (n_walkers).  Any may
 * be NULL.  Host pointers; synchronises. */
afqmc_status afqmc_get_walkers(afqmc_sys sys, double* phi, double* w, double* log_ovlp,
                               unsigned char* alive);

/* Query sizes: any pointer may be NULL. */
afqmc_status afqmc_sys_info(afqmc_sys sys, int* M, int* n_chol, int* n_alpha, int* n_beta,
                            int* n_walkers, int64_t* step);

/* Snapshot of the walker state (phi, weights, overlaps, Theta as the step
 * stores it (FP64 for AFQMC_FP64, else the FP32/BF16 copy), alive, step
 * counter).  dst NULL: *bytes receives the size needed.  Restoring a snapshot
 * and stepping again with the same seed reproduces the original run bit for
 * bit (the fields are a pure function of the step counter). */
afqmc_status afqmc_checkpoint(afqmc_sys sys, void* dst, size_t* bytes);
afqmc_status afqmc_restore(afqmc_sys sys, const void* src, size_t bytes);

void afqmc_free_sys(afqmc_sys sys);
void afqmc_free_ham(afqmc_ham ham);

/* Thread-local message describing the last non-OK status of this thread. */
const char* afqmc_last_error(void);

/* Per-phase kernel timing with HIP events on the system's stream.
 * afqmc_profile_enable(sys, 1) clears the counters and starts recording a
 * start/stop event pair around every kernel launch of every later step
 * (phases: 0 force-bias GEMM, 1 fields, 2 field-sum GEMM, 3 unpacking of
 * the symmetric A, 4 fused propagation P T_K(A) P, 5 overlaps, determinants
 * and Theta, 6 weights, 7 Gram-Schmidt, 8 exchange (one launch per spin),
 * 9 local/mixed energy); 0 stops.  afqmc_profile_read
 * synchronises and returns the summed milliseconds and the launch count of
 * one phase.  afqmc_phase_name returns a phase's name, NULL past the last. */
afqmc_status afqmc_profile_enable(afqmc_sys sys, int enable);
afqmc_status afqmc_profile_read(afqmc_sys sys, int phase, double* total_ms, int64_t* launches);
const char* afqmc_phase_name(int phase);

/* Kernel self-test: C = A * B^T (A: m x k, B: n x k, C: m x n, host
 * float64) computed by the library's tiled MFMA GEMM in precision `prec`
 * (inputs rounded to that precision).  For the numerics tests of the
 * contraction kernel against a plain reference.  Synchronises. */
afqmc_status afqmc_selftest_gemm(afqmc_prec prec, int m, int n, int k, const double* A,
                                 const double* B, double* C);

/* Kernel self-test with the launch shape fixed: C = A * B^T as above, with
 * the operands held in the storage the walker step gives its contractions
 * (FP64 for AFQMC_FP64; FP32 for AFQMC_FP32 and for AFQMC_BF16, which here
 * selects the split-BF16 products) and an FP64 result.  tile: 0 size
 * heuristic, 1 64 x 64, 2 128 x 128, 3 256 x 128 workgroup tiles, 4 256 x 128
 * over 16 wavefronts (split BF16; the others as 3); ksplit
 * >= 1: K cut into that many ranges whose partial sums are added in range
 * order.  Every tile shape gives the same bits for the same ksplit.  For the
 * tests of the GEMM paths the walker step takes.  Errors: E_INVALID.
 * Synchronises. */
afqmc_status afqmc_selftest_gemm_shape(afqmc_prec prec, int tile, int ksplit, int m, int n, int k,
                                       const double* A, const double* B, double* C);

/* Kernel self-test of the fused propagation: out[w] = P T_K(A_w) P phi[w]
 * (Eq. 3 and Eq. 11, T_K the order-K Taylor polynomial of exp) with the
 * products in precision `prec` (AFQMC_FP64; AFQMC_BF16X3: Taylor terms and
 * P - I in split BF16, the identity part of P added in FP32; else FP32), workgroup shape `variant` (waves x
 * column blocks per wave: 0: 8 x 2, 1: 4 x 2, 2: 4 x 1, 3: 2 x 2, with the
 * next chunk of the matrix operand prefetched; 4..7: the same shapes without
 * the prefetch, FP32 and split BF16 only; 8: 16 x 1, 9: 8 x 1, 10: 8 x 2 and
 * 11: 4 x 2 with two row blocks (32 orbitals) per workgroup, split BF16
 * only (8, 9 keep the running Taylor sum in LDS); 12: 8 x 2 and 13: 16 x 1
 * with five row blocks (80 orbitals) per workgroup, split BF16 and M rounded
 * up to 32 at most 224 only; a shape serves M <= 16 waves blocks; E_SHAPE
 * otherwise).
 * phi, out:
 * nw x 2 x N x M (plane 0 real, plane 1 imaginary of orbital columns); P:
 * M x M real symmetric; A: nw x 2 x M x M complex symmetric.  Host float64
 * arrays; synchronises.  For the numerics tests of the propagation kernel. */
afqmc_status afqmc_selftest_propagate(afqmc_prec prec, int M, int N, int nw, int K, int variant,
                                      const double* phi, const double* P, const double* A,
                                      double* out);

/* Device Philox4x32-10 normals x[k, gamma] of step t for walkers 0..nw-1,
 * the same values afqmc_step draws; host output nw x n_chol.  For tests. */
afqmc_status afqmc_selftest_fields(uint64_t seed, uint64_t stream_id, int64_t t, int nw,
                                   int n_chol, double* out);

#ifdef __cplusplus
}
#endif

#endif /* AFQMC_H */
