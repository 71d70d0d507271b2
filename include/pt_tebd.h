/*
 * pt_tebd.h -- C ABI of the MI355X PT-TEBD library (libpt_tebd.so).
 *
 * PT-TEBD (Fux, Kilda, Lovett, Keeling, arXiv 2201.05529) propagates the
 * vectorised density matrix of a chain of open quantum systems as an
 * "augmented" MPS whose site tensors carry one extra leg per bath: the bond
 * of that bath's process-tensor MPO (PT-MPO).  One time step absorbs the
 * PT-MPO tensor of every bath site and applies two-site Liouville-space
 * propagators on the chain bonds (Sec. II.A; Appendix A).
 *
 * Problem statement (Appendix A, eq. total-hamiltonian): H = sum_n (H^S_n +
 * H^E_n) + sum_n K_{n,n+1}, each environment H^E_n coupled to one site only,
 * optional on-site GKSL terms (Appendix A.1).  The environments enter only
 * through precomputed PT-MPOs (Appendix A.1, Fig. tensor-network-
 * construction (b)); pt_mpo_build_ohmic() builds one for a Gaussian bath.
 *
 * Conventions shared by every call:
 *  - complex numbers are interleaved (re, im) doubles; arrays are row-major;
 *    sites are 0-based;
 *  - Liouville index of one site: s = i*d + j for rho_ij (row-major vec);
 *  - two-site operators K_{n,n+1} are given in the natural two-site order,
 *    row (i_n i_{n+1}), column (j_n j_{n+1});
 *  - the library copies every input it is given; the caller keeps ownership
 *    of all its pointers and of the device workspace, which must outlive
 *    the handle;
 *  - no call throws; every call returns a status.  Errors found on the
 *    device (non-finite numbers, a zero norm) are sticky per handle and are
 *    reported by the next call that synchronises (observe, correlate,
 *    bond_dims, snapshot); pt_tebd_last_error() gives a message.
 *  - one host thread per handle at a time.  Work is enqueued on the HIP
 *    stream given at creation; calls that return host data synchronise it.
 */
#ifndef PT_TEBD_H
#define PT_TEBD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pt_tebd* pt_tebd_t;

typedef enum {
  PT_TEBD_OK = 0,
  PT_TEBD_EINVAL = -1,   /* invalid argument or configuration              */
  PT_TEBD_ENOMEM = -2,   /* workspace too small                              */
  PT_TEBD_EDEVICE = -3,  /* a HIP runtime call failed                        */
  PT_TEBD_ENUMERIC = -4, /* non-finite value or zero norm met on the device  */
  PT_TEBD_ENOCONV = -5,  /* an iterative eigensolver stage did not converge  */
  PT_TEBD_ERANGE = -6    /* stepped past the end of a PT-MPO, or a size read
                            on the device exceeded its workspace (internal) */
} pt_tebd_status;

typedef enum {
  PT_TEBD_FP64 = 0,       /* every contraction in double precision (matrix
                             cores, v_mfma_f64)                              */
  PT_TEBD_FP32_MIXED = 1  /* the contractions that form D (Appendix A.2
                             (e)-(f)), the range finder's products with D and
                             the rebuild of the site tensors ((g)-(h)) in
                             single precision on the matrix cores (real-split
                             complex products, single-precision accumulation);
                             Gram matrices, eigensolvers, singular values,
                             lambda, the gate, the PT absorption, the
                             log-scale and the read-out in double.  The
                             truncation additionally discards singular values
                             below u_32 ||X||_F (the single-precision noise
                             floor of the contracted matrix X).              */
} pt_tebd_precision;

/* One bath: a PT-MPO attached to one site (Appendix A.1).  Tensor k
 * (k = 1..n_steps) is P_k[e][e'][s_out][s_in] with e of dimension
 * bond_dims[k-1] and e' of dimension bond_dims[k]; with diagonal = 1 (the
 * coupling operator is diagonal in the computational basis) it is
 * P_k[e][e'][s].  bond_dims[0] must be 1 (uncorrelated initial state).
 * caps[k] (k = 0..n_steps) is the cap vector of step k (Appendix A.3) of
 * length bond_dims[k]; caps = NULL makes the library compute them by the
 * backward recursion (trace the output, feed the maximally mixed input). */
typedef struct {
  int32_t site;
  int32_t n_steps;
  const int32_t* bond_dims;      /* [n_steps + 1]                      */
  int32_t diagonal;
  const double* const* tensors;  /* [n_steps] pointers, complex        */
  const double* const* caps;     /* [n_steps + 1] pointers or NULL     */
  /* Initially correlated chain site and environment (Appendix A.1: the
   * augmented legs of the initial MPS have dimension > 1): with
   * bond_dims[0] > 1, the bath site's initial augmented tensor R[s][e],
   * complex [d^2][bond_dims[0]] (s the site's Liouville index i d + j of
   * rho_ij, e the PT-MPO's first bond), which replaces that site's rho0.
   * NULL (an uncorrelated start) requires bond_dims[0] = 1. */
  const double* initial;
} pt_tebd_bath;

typedef struct {
  int32_t n_sites;               /* N >= 1                                    */
  int32_t d;                     /* local Hilbert dimension; must be 2        */
  double dt;                     /* full time step, > 0                       */
  const double* h_site;          /* [N][d][d] complex, Hermitian: H^S_n       */
  const double* h_bond;          /* [N-1][d*d][d*d] complex, Hermitian: K     */
  int32_t n_lindblad;            /* GKSL operators per site (may be 0)        */
  const double* lindblad;        /* [N][n_lindblad][d][d] complex or NULL     */
  const double* rho0;            /* [N][d][d] complex: product initial state  */
  int32_t n_baths;               /* at most one bath per site                 */
  const pt_tebd_bath* baths;
  int32_t chi_max;               /* cap of the chain bond dimension           */
  int32_t xi_max;                /* >= every PT-MPO bond dimension            */
  double svd_rel_cutoff;         /* eps of the truncation rule (Appendix A.2) */
  pt_tebd_precision precision;
  uint64_t seed;                 /* seed of the randomised range finder       */
} pt_tebd_config;

/* Device workspace (bytes) a handle needs for cfg. */
pt_tebd_status pt_tebd_workspace_size(const pt_tebd_config* cfg, size_t* bytes);

/* Validate cfg, build the chain propagators (Appendix A.1: on-site terms
 * absorbed into the bonds, second-order even/odd splitting, gates
 * exp(L^{K'} dt/4) and the merged dt/2 gates), copy the PT-MPOs and the
 * initial product state (Vidal form with dummy augmented legs, Appendix A.1)
 * into the caller's device workspace, and return a handle.  hip_stream is a
 * hipStream_t (NULL = default stream). */
pt_tebd_status pt_tebd_create(const pt_tebd_config* cfg, void* dev_workspace, size_t bytes,
                              void* hip_stream, pt_tebd_t* out);

/* Enqueue n_steps time steps (eq. propagator-env): each is a chain half-step
 * E(dt/4) O(dt/2) E(dt/4), the absorption of P_k on every bath site
 * (Appendix A.2 (i)-(j)), and another chain half-step.  Each two-site gate
 * uses the contraction and truncated-SVD sequence of Appendix A.2 (c)-(h).
 * Asynchronous; returns PT_TEBD_ERANGE if the PT-MPOs are too short. */
pt_tebd_status pt_tebd_step(pt_tebd_t h, int32_t n_steps);

/* <O_i> = Tr[O_i rho] / Tr rho at the current step for n_ops single-site
 * operators (ops: [n_ops][d][d] complex, sites: [n_ops]) via the caps of the
 * current step (Appendix A.3, Fig. tensor-network-contraction (k)-(l)).
 * out: [n_ops] complex.  trace_out (complex Tr rho, may be NULL).  Syncs. */
pt_tebd_status pt_tebd_observe(pt_tebd_t h, int32_t n_ops, const int32_t* sites,
                               const double* ops, double* out, double* trace_out);

/* Two-time correlation (Appendix A.4, eq. two-time-corr-decomposed):
 * out[j] = Tr[B X(t + j dt)] / Tr rho(t), j = 0..n_steps, where X(t) = A rho(t)
 * (A acting on site_a from the left) is propagated from a device copy of the
 * full augmented state.  The handle's own state is not changed.  Syncs. */
pt_tebd_status pt_tebd_correlate(pt_tebd_t h, int32_t site_a, const double* op_a,
                                 int32_t site_b, const double* op_b, int32_t n_steps,
                                 double* out);

/* Multi-time correlation (Appendix A.4, eq. two-time-corr-decomposed with P
 * insertions): from the current step t a device copy X of the augmented
 * state is propagated; at step offset offsets[p] (non-decreasing, >= 0) the
 * super-operator of ops[p] (complex 2x2, row-major) acts on site sites[p],
 * from the left (sides[p] = 0: C rho, the C^L of the paper) or from the
 * right (sides[p] = 1: rho C, the C^R of out-of-time-ordered correlations).
 * out[j] = Tr[B X(t + (m_P + j) dt)] / Tr rho(t), j = 0..n_steps, m_P the
 * last offset (complex, interleaved).  pt_tebd_correlate is the case of one
 * left insertion at offset 0.  The handle's own state is not changed.
 * EINVAL for offsets out of order, sides other than 0 or 1, sites out of
 * range or non-finite operators; ERANGE when the propagation runs past a
 * PT-MPO.  Syncs. */
pt_tebd_status pt_tebd_correlate_multi(pt_tebd_t h, int32_t n_ins, const int32_t* offsets, const int32_t* sites,
                                       const double* ops, const int32_t* sides, int32_t site_b, const double* op_b,
                                       int32_t n_steps, double* out);

/* Fluctuation and dissipation spectra of a Hermitian single-site operator A
 * at the current (steady) state, Sec. III.A and Appendix B.2: the
 * auto-correlation C(tau_j) = <A(tau_j) A(0)> = Tr[A X(t + tau_j)] / Tr rho(t)
 * with X(t) = A rho(t), tau_j = j dt, j = 0..n_steps, goes to corr (complex,
 * interleaved, n_steps + 1 values).  Continued to negative times by
 * C(-tau) = C(tau)^* and transformed on [-n_steps dt, n_steps dt] with the
 * trapezoid rule at the n_omega angular frequencies omega:
 *   s_out[k]   = S_A(w)   = dt sum_j c_j Re C(tau_j) cos(w tau_j)
 *   chi_out[k] = chi''_A(w) = -dt sum_j c_j Im C(tau_j) sin(w tau_j)
 * with c_0 = c_n = 1 and c_j = 2 otherwise, so S_A is the transform of
 * 1/2 <{A(tau), A(0)}> and chi''_A the imaginary part of the transform of
 * i Theta(tau) <[A(tau), A(0)]>.  For a thermal state at temperature T,
 * S_A / chi''_A = coth(w / 2T).  The transform runs on the device (one
 * thread per frequency); the call allocates and frees small device buffers
 * and syncs.  EINVAL for a non-Hermitian A. */
pt_tebd_status pt_tebd_fdt_spectra(pt_tebd_t h, int32_t site, const double* op, int32_t n_steps, int32_t n_omega,
                                   const double* omega, double* corr, double* s_out, double* chi_out);

/* Current chain bond dimensions chi[N-1] and augmented dims xi[N] (xi may be
 * NULL).  Syncs. */
pt_tebd_status pt_tebd_bond_dims(pt_tebd_t h, int32_t* chi, int32_t* xi);

/* Minimal algorithmic work of the bond updates stepped so far, from the run-
 * time dims of every update (chi_{n-1}, xi_n, chi_n, xi_{n+1}, chi_{n+1},
 * the ranks l, r of B_L, B_R and the new chi'), in flops with a complex
 * multiply-add counted as 8 (Appendix A.2 (c)-(h)):
 *   out[0] F_a1 = 16 (chi_{n-1} xi_n)(d^2 chi_n) l + 16 (d^2 chi_n)(xi_{n+1} chi_{n+1}) r
 *               (rank-l / rank-r factorisations of B_L and B_R, two passes)
 *   out[1] F_a2 = 8 (d^2 l) chi_n (d^2 r) + 8 d^8 l r   (X lambda Y and the gate)
 *   out[2] F_a3 = 16 (d^2 l)(d^2 r) chi'                   (top-chi' part of D)
 *   out[3] F_a4 = 8 (chi_{n-1} xi_n) l (d^2 chi') + 8 (d^2 chi') r (xi_{n+1} chi_{n+1})
 *               (the two rebuild products)
 * Counted on the device in each update's final kernel; reset != 0 clears
 * the counters after the read.  Syncs. */
pt_tebd_status pt_tebd_model_flops(pt_tebd_t h, double* out, int32_t reset);

/* Host copy of the whole augmented state (Gamma, lambda, log-scale, step).
 * With buf = NULL only *bytes is set.  Syncs.  pt_tebd_restore loads it back
 * into a handle created from the same configuration: EINVAL (nothing is
 * copied) when bytes is shorter than a snapshot of this handle, when the
 * header does not match the handle, or when the stored step lies outside
 * [0, PT-MPO length]; on success the handle's sticky error state is cleared. */
pt_tebd_status pt_tebd_snapshot(pt_tebd_t h, void* buf, size_t* bytes);
pt_tebd_status pt_tebd_restore(pt_tebd_t h, const void* buf, size_t bytes);

int32_t pt_tebd_current_step(pt_tebd_t h);
/* Message of the handle's last error; with h == NULL, the message of the
 * last failed pt_tebd_create on the calling thread.  The string is owned by
 * the library and valid until the next call on the same handle (thread). */
const char* pt_tebd_last_error(pt_tebd_t h);
void pt_tebd_destroy(pt_tebd_t h);

/* Batches: many chains advanced together (the bond updates of a sublayer
 * are independent, Sec. II.B and Appendix A.2, across chains as within
 * one).  Each kernel of a sublayer runs once over the bond updates of every
 * chain of the batch, the PT absorption once over every (chain, bath) pair,
 * and one time step is captured in a HIP graph on first use and replayed.
 * The handles must share one stream (not the NULL stream for the graph; on
 * the NULL stream the launches are issued directly), the precision and the
 * truncation settings, and have at least two sites; chains may differ in
 * length, bond caps and PT-MPOs, and may be at different steps.  The batch
 * keeps pointers to the handles: destroy it before any of them.  While a
 * batch exists, pt_tebd_step on a member (or a restore) is allowed; the
 * batch reads each handle's current step when it starts stepping.
 * pt_tebd_batch_workspace_size gives the device bytes of the batch's job
 * tables; the caller owns that workspace, which must outlive the batch. */
typedef struct pt_tebd_batch* pt_tebd_batch_t;
pt_tebd_status pt_tebd_batch_workspace_size(pt_tebd_t* hs, int32_t n, size_t* bytes);
pt_tebd_status pt_tebd_batch_create(pt_tebd_t* hs, int32_t n, void* dev_workspace, size_t bytes,
                                    pt_tebd_batch_t* out);
/* Enqueue n_steps time steps of every chain (asynchronous; ERANGE if a chain
 * would pass the end of its PT-MPO, nothing enqueued then).  Device-side
 * errors are sticky per chain and reported by that handle's next syncing
 * call. */
pt_tebd_status pt_tebd_batch_step(pt_tebd_batch_t b, int32_t n_steps);
const char* pt_tebd_batch_last_error(pt_tebd_batch_t b);  /* NULL: last failed batch_create */
void pt_tebd_batch_destroy(pt_tebd_batch_t b);

/* Advance n handles by n_steps time steps each as one batch (above), with
 * the batch's job tables in device memory allocated and freed by the call
 * (hipMalloc); synchronises before returning. */
pt_tebd_status pt_tebd_step_many(pt_tebd_t* hs, int32_t n, int32_t n_steps);

/* Measurement support (not part of the method).  pt_tebd_kernel_timing
 * selects one kernel class (0 none, 1 the batched eigensolver's solve kernel,
 * 2 the batched complex GEMM of the bond update) and resets the counters;
 * while set, every launch of that class made by pt_tebd_step or
 * pt_tebd_correlate on this handle is bracketed by HIP events on the
 * handle's stream, and the kernels add their algorithmic flop counts
 * (16 n^3 / 3 per n x n Hermitian tridiagonal reduction; 8 m n k per complex
 * m x n x k product) to a device counter.  pt_tebd_kernel_timing_read
 * synchronises and returns the summed event time (ms), the number of
 * launches and the flop count since the last reset.  EINVAL for a bad
 * class or null pointers. */
pt_tebd_status pt_tebd_kernel_timing(pt_tebd_t h, int32_t kernel_class);
pt_tebd_status pt_tebd_kernel_timing_read(pt_tebd_t h, double* total_ms, int64_t* launches,
                                          double* alg_flops);

/* Host helper (not on the hot path): PT-MPO of a Gaussian bosonic bath with
 * J(w) = 2 alpha w exp(-w/wc) (cutoff_kind 0) or 2 alpha w exp(-w^2/wc^2)
 * (cutoff_kind 1) at temperature T coupled through the d x d Hermitian
 * operator coupling_op (complex), for time step dt, n_steps steps, memory
 * cutoff mem_steps (Appendix B.1: Delta K_max) and truncation threshold eps
 * (eps_TEMPO) with bond cap xi_max.  The influence functional is discretised
 * for piecewise-constant system paths and compressed forward in time.
 * out->tensors and out->bond_dims are allocated by the library; free them
 * with pt_mpo_free.  out->caps is NULL. */
pt_tebd_status pt_mpo_build_ohmic(double alpha, double wc, int32_t cutoff_kind, double temperature,
                                  double dt, int32_t n_steps, int32_t mem_steps, double eps,
                                  int32_t xi_max, const double* coupling_op, int32_t d,
                                  pt_tebd_bath* out);
void pt_mpo_free(pt_tebd_bath* bath);

/* The same PT-MPO construction (Appendix B.1) for n_builds baths at once on
 * the GPU: every bath is one work item of the batched window sweeps (right
 * to left LQ factorisations, left to right truncated SVDs through Gram
 * matrices and the double-precision eigensolver).  params[b] gives alpha,
 * wc, temperature, cutoff_kind, the coupling operator and the length of
 * bath b's PT-MPO (a build of M steps equals the single build of M steps:
 * builds advance in lockstep and one of them stops at its own length); dt,
 * mem_steps, eps and xi_max (<= 256) are shared, n_steps is the longest.  out[b] is filled
 * as by pt_mpo_build_ohmic (library-owned host arrays, free each with
 * pt_mpo_free).  Device memory (about (mem_steps + 6) (4 xi_max)^2 * 64 B
 * plus n_steps xi_max^2 * 64 B per bath) is allocated and freed by the call;
 * work runs on hip_stream, and the call synchronises it. */
typedef struct {
  double alpha, wc, temperature;
  int32_t cutoff_kind;
  const double* coupling_op;   /* d x d Hermitian, complex */
  int32_t n_steps;             /* this bath's PT-MPO length, 1..n_steps of the call; 0: the call's n_steps */
} pt_bath_params;
pt_tebd_status pt_mpo_build_ohmic_batch(int32_t n_builds, const pt_bath_params* params, double dt,
                                        int32_t n_steps, int32_t mem_steps, double eps, int32_t xi_max,
                                        int32_t d, void* hip_stream, pt_tebd_bath* out);

/* eta_Delta (Delta = 0..mem_steps) of the same discretisation, complex
 * [mem_steps + 1]; exposed for testing. */
pt_tebd_status pt_bath_eta(double alpha, double wc, int32_t cutoff_kind, double temperature,
                           double dt, int32_t mem_steps, double* eta_out);

/* The site-major two-site propagator of bond b (complex [d^4][d^4]) that
 * pt_tebd_create built; exposed for testing.  Host-side, no sync. */
pt_tebd_status pt_tebd_gate(pt_tebd_t h, int32_t bond, double* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * Hermitian eigensolver of the truncated SVDs with no allocation at all.
 * n x n complex Hermitian a_dev (row-major, interleaved (re, im), n <= 256,
 * caller-owned device memory, not modified), rule as pt_test_heev (0 every
 * positive eigenvalue, 1 the eps rule on sqrt(eigenvalues), 2 the eps rule
 * plus the cap, 3 numerical rank lambda_k > eps lambda_0, 4 every
 * eigenpair).  Outputs, all caller-owned device memory: w_dev [n]
 * eigenvalues (descending), v_dev [n][n] complex with the selected vectors
 * in columns 0..nvec-1 (the other columns are left as they were),
 * nvec_dev [1], status_dev [1] (the eigensolver's error word, 0 = OK).
 * Every other buffer lives in one static device array of the library
 * (about 6.6 MB per GPU, held until the process ends), so the call makes no
 * hipMalloc, hipFree or allocating library call; it only enqueues kernels
 * on hip_stream (NULL = default stream) and returns without synchronising.
 * Calls that overlap on one GPU share that array and race: serialise them
 * (one stream, or events).  EINVAL for n outside [1, 256], a bad rule or a
 * null pointer; EDEVICE if a launch fails. */
pt_tebd_status pt_heev_noalloc(int32_t n, const double* a_dev, int32_t rule, double eps, int32_t cap,
                               double* w_dev, double* v_dev, int32_t* nvec_dev, int32_t* status_dev,
                               void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* PT_TEBD_H */
