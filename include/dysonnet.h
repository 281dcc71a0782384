/*
 * dysonnet.h -- C ABI of the MI355X (gfx950) DysonNet local-estimator library.
 *
 * What it computes (paper: "DysonNet: Constant-Time Local Updates for Neural Quantum
 * States"): for a batch of spin configurations s[B,N] it evaluates log psi(s) with a
 * DysonNet (Sec. II, Eq. (wavefunc); S4 Green's-function mixers, Sec. V and App.
 * "Details on the implementation of the DysonNet block"), the log-amplitude ratio
 * log psi(s')/psi(s) of every connected configuration s' of a Hamiltonian -- either by
 * the ABACUS local update (Sec. III, Algorithm 1, Eqs. (recur_step)-(recur_out),
 * Theorem 1) or by full re-evaluation -- and the local energy
 * E_loc(s) = sum_s' <s|H|s'> psi(s')/psi(s) (Eq. (local-estimator)).
 *
 * Conventions shared by every call
 *  - Every function returns dn_status (0 = DN_OK). On failure nothing is promised about
 *    the outputs; dn_last_error() returns a thread-local message.
 *  - Array arguments are DEVICE pointers unless stated otherwise. The caller allocates
 *    and owns them; the library never frees them. All calls are asynchronous on the
 *    given stream (a hipStream_t passed as void*; NULL = the default stream); outputs
 *    are valid once the stream has synchronised.
 *  - The library owns each model: its parameters, the derived tables (Green's-function
 *    taps, transposed weights) and a growable workspace. A model must not be used from
 *    two streams at the same time.
 *  - spins: int8, values +1/-1, row-major [B, N]. dn_logratio and dn_eloc reject other
 *    values with DN_EINVAL (checked on the device with the work list, before any network
 *    kernel runs); the calls without a work list (dn_logpsi, dn_grad_logpsi, the sampler,
 *    the ragged batch) do not check them and give undefined results for them.
 *  - sites: int32 [B, M_max, 2]; element m of sample b flips sites[b,m,0] and, unless it
 *    is -1, sites[b,m,1]. Entries m >= n_conn[b] are ignored on input.
 *  - logpsi, logratio, eloc, helem, hdiag are float64 in every precision mode. For a model
 *    with complex_out = 1, logpsi, logratio and eloc hold complex values instead: (re, im)
 *    float64 pairs, i.e. logpsi [B][2], logratio [B, M_max][2], eloc [B][2] (the layout of
 *    C99 double complex); a phase is reported in [-pi, pi].
 */
#ifndef DYSONNET_H
#define DYSONNET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DN_OK = 0,
  DN_EINVAL = 1,        /* bad argument: shape, enum, null pointer, M_max too small */
  DN_ENOMEM = 2,        /* device allocation failed or the workspace limit was hit */
  DN_EHIP = 3,          /* a HIP runtime call failed */
  DN_EUNSUPPORTED = 4,  /* valid request outside what the kernels implement */
  DN_ESTATE = 5         /* call out of order (e.g. no parameters set yet) */
} dn_status;

typedef enum { DN_BC_OPEN = 0, DN_BC_PERIODIC = 1 } dn_bc;
typedef enum { DN_ACT_SILU = 0, DN_ACT_TANH = 1, DN_ACT_IDENTITY = 2 } dn_act;
/* Arithmetic of the network fields and channel mixing. FP64: everything float64.
 * FP32: float32 fields, float32 MFMA with float32 accumulation; the Green's-function
 * (Toeplitz) products and the ABACUS deep blocks' channel mixing by default on the bf16
 * matrix cores with both float operands split into three bf16 terms, which keeps float32
 * accuracy (see dn_set_product_mode). BF16_MIXED (d > 16): the
 * two channel-mixing products of every block (V and U: forward, adjoint and the ABACUS
 * propagation) run on the bf16 matrix cores with float32 accumulation, each operand split
 * into hi + lo bfloat16 terms (round to nearest even; 16 significant bits) and the three
 * partial products hi*hi, hi*lo, lo*hi accumulated (relative error of a product below
 * 3 * 2^-17), and so do the Green's-function (Toeplitz) products (hi + lo terms of both the
 * field and the taps); everything else as FP32 (phi stream, slices, the per-flip update of
 * one- and two-block networks; per-sample gradients run entirely in float32). Kernel
 * generation, the read-out sums and the log-ratio are float64 in every mode. */
typedef enum { DN_PREC_FP64 = 0, DN_PREC_FP32 = 1, DN_PREC_BF16_MIXED = 2 } dn_prec;
typedef enum { DN_PATH_ABACUS = 0, DN_PATH_FULL = 1 } dn_path;

/* Network hyper-parameters (Sec. II; App. "Details on the implementation ...").
 * N chain length in tokens (network sites); L blocks; d channels (d <= 64); s S4 state size (s <= 32);
 * d_out log-cosh read-out units (must be 2); w_c half-width of the phi-stream CNN
 * (0..3); bc network boundary condition (dn_bc); act local nonlinearity g (dn_act);
 * inject_phi 1 adds phi^(l) to the h stream before each mixer (Fig. 1c form);
 * prec arithmetic (dn_prec); complex_out 1 makes the read-out matrix A complex (Sec. II: a
 * complex A gives a complex wavefunction): its two columns are Re A and Im A, the two
 * pre-activations form one complex unit Omega = Omega_0 + i Omega_1 and
 * log psi = log cosh(Omega) is complex (0: two real units, log psi = sum_k log cosh Omega_k);
 * token spins per token (patching, Sec. V; 0 or 1 = one spin per site, at most 4): token tau
 * holds spins token*tau .. token*tau + token - 1 and is embedded as sum_k E_k s_(token*tau + k),
 * likewise the phi stream with E_phi,k. Spin arrays then hold N * token spins per sample and
 * sites index spins; a flip changes one token, a pair exchange one token or two;
 * d_block > 0 makes the vertex D = U diag(chi) V block-diagonal in channel blocks of d_block
 * (Sec. V, the mixture-of-experts remark; d_block divides d): the off-block entries of U and V
 * in the parameter vector are not used and get zero log-derivatives. */
typedef struct {
  int32_t N, L, d, s, d_out, w_c;
  int32_t bc, act, inject_phi, prec;
  int32_t complex_out, token, d_block;
} dn_model_desc;

typedef enum { DN_H_LRTFIM = 0, DN_H_J1J2 = 1 } dn_ham_kind;

/* Hamiltonian. DN_H_LRTFIM (Sec. VI): paper_form = 0 gives
 *   H = sum_{i<j} J sz_i sz_j / dist^alpha + h sum_i sx_i,
 * paper_form = 1 gives H = -(J/N_alpha) sum_{i!=j} sz sz / dist^alpha - h sum sx with
 * N_alpha = 2 sum_{r=1}^{floor(N/2)} r^-alpha; dist = |i-j| (bc open) or
 * min(|i-j|, N-|i-j|) (periodic). Connected elements: the N single flips, m = site.
 * DN_H_J1J2 (Eq. (j1j2_hamiltonian), S = sigma/2): J1 on bonds (i,i+1), J2 on (i,i+2);
 * diagonal (J/4) s_i s_j per bond, element J/2 per antiparallel bond, emitted in the
 * order i = 0..N-1, then delta = 1, 2 (bonds leaving an open chain are skipped); N >= 5. */
typedef struct {
  int32_t kind, bc;
  double J, alpha, h;
  int32_t paper_form;
  double J1, J2;
} dn_ham_desc;

typedef struct dn_model dn_model; /* opaque */

/* Length of the flat float64 parameter vector for this shape (-1 if the shape is
 * invalid). Order: E[token][d], E_phi[token][d]; per block: W_D[d,d], w[d], K[2w_c+1,d], k[d],
 * A_D[d,d], b[d], U[d,d], V[d,d]; per mixer (blocks 1..L then the final mixer), per
 * channel: 12 vectors of length s (Lambda raw real part, Lambda imaginary part, p re/im,
 * q re/im, B re/im, C+ re/im, C- re/im) and one step offset; A[d, d_out]. Matrices are
 * row-major, output index first. Lambda = -exp(raw) + i*raw';
 * Delta_c = exp(ln 0.01 + ln 10 * c/(d-1) + offset_c). */
int64_t dn_param_count(const dn_model_desc* desc);

/* Create a model (no parameters yet). Validates the shape; DN_EUNSUPPORTED for shapes
 * the kernels do not cover (d > 64, s > 32, d_out != 2, N > 512, a float64 field of one
 * configuration larger than the on-chip tile, or BF16_MIXED with d <= 16). *out receives
 * the handle. */
dn_status dn_model_create(const dn_model_desc* desc, dn_model** out);

/* Cap the workspace the model may allocate (bytes; 0 = no cap). Calls that would need
 * more fail with DN_ENOMEM. */
dn_status dn_set_workspace_limit(dn_model* m, size_t bytes);

/* Copy the flat float64 parameter vector (host pointer if params_on_device == 0, else
 * device) and derive every parameter-only table on the GPU: S4 Green's-function taps of
 * every mixer by bilinear discretisation and state-matrix powers in float64 (Sec. V,
 * Eq. (discretization)), transposed/padded weight copies, read-out weights. Synchronises
 * the stream once to check that the taps are finite (DN_EINVAL otherwise). */
dn_status dn_model_set_params(dn_model* m, const double* params, int params_on_device, void* stream);

/* Copy the float64 Green's-function taps to taps_out (device), layout [L+1][d][2N-1],
 * offset r = i - i' stored at r + N - 1 (periodic: the aliased kernel g_(r mod N)). */
dn_status dn_model_get_taps(dn_model* m, double* taps_out, void* stream);

/* log psi(s) for B configurations (Eq. (wavefunc) with f = log cosh). Asynchronous on the
 * stream. */
dn_status dn_logpsi(dn_model* m, const int8_t* spins, int32_t B, double* logpsi, void* stream);

/* One half-sweep of the screened typewriter Metropolis sampler over B independent chains
 * (Sec. IV, Algorithm 2; App. "Screened Metropolis sampler is exact"; App. "Practical
 * implementation of the screened typewriter sampler"). The chain is cut into blocks of
 * `spacing` sites; the visited blocks are b = parity, parity + 2, ... (K = (ceil(N / spacing)
 * - parity + 1) / 2 of them, in that order) and block b proposes flipping site
 * b*spacing + floor(r * width), width = min(spacing, N - b*spacing). The proposals' output changes
 * come from ABACUS against one background; proposal k is judged with the independent-scattering
 * ratio R~ = prod_units cosh^2(Omega + dOmega_k) / cosh^2(Omega), Omega accumulating the
 * accepted changes. A draw with |u - min(1, R~)| <= eps freezes the chain there: its background
 * is rebuilt at its current configuration and the remaining proposals recomputed, the frozen
 * one then decided with its exact ratio; otherwise accept iff u < min(1, R~). When eps bounds
 * |R~ - R| the decisions are exact Metropolis-Hastings decisions for the same draws.
 * spins: device int8 [B][N], updated in place. r_site, u: device float64 [B][K] (uniform draws
 * in [0, 1), supplied by the caller). accepted: device int32 [B][K] (1 = accepted); refreshes:
 * device int32 [B] (background rebuilds per chain). The sampler's ABACUS uses the model's
 * workspace; one host synchronisation per refresh round. Requirements as for DN_PATH_ABACUS.
 * A two-block network with at most 32 proposals per chain propagates each proposal through
 * block 1 over the whole chain instead of building block 2's pivot-0 link per chain (cheaper
 * at so few flips per background; same results). */
dn_status dn_screened_sweep(dn_model* m, int8_t* spins, int32_t B, int32_t spacing, int32_t parity,
                            const double* r_site, const double* u, double eps, int32_t* accepted,
                            int32_t* refreshes, void* stream);

/* dn_screened_sweep with the practical tolerance schedule of App. "Practical implementation of
 * the screened typewriter sampler": a proposal is screened with eps_buf[min(n, n_eps - 1)], n
 * the flips accepted since the chain's current background. Every refresh records the frozen
 * proposal's empirical error e~ = |min(1, R~) - min(1, R)| (R its exact ratio at the refreshed
 * background) with the n at which the chain froze. After the half-sweep the events are applied
 * to the buffer, chain by chain in chain order and in order within a chain: an entry whose
 * eps_set flag is 0 (still at the caller's default) takes e~ and its flag becomes 1; any other
 * becomes max(entry, gamma e~). eps_buf (device float64 [n_eps]) and eps_set (device int32
 * [n_eps]) are the caller's, updated in place and shared by all chains of the call; the buffer
 * is fixed while the half-sweep runs. gamma >= 1 (the paper takes gamma > 1). Other arguments,
 * outputs and requirements as for dn_screened_sweep. */
dn_status dn_screened_sweep_adaptive(dn_model* m, int8_t* spins, int32_t B, int32_t spacing, int32_t parity,
                                     const double* r_site, const double* u, double* eps_buf, int32_t* eps_set,
                                     int32_t n_eps, double gamma, int32_t* accepted, int32_t* refreshes,
                                     void* stream);

/* One stochastic-reconfiguration (natural-gradient) update of variational Monte Carlo (Sec. II
 * and VI; App. "Network parameters": standard SR with a diagonal shift). Inputs: the per-sample
 * log-derivatives O [B][P] as dn_grad_logpsi writes them (device, the model's field type: float
 * for FP32 / BF16-mixed models, double for FP64), local energies eloc [B] (device float64) and
 * sample weights [B] (device float64 summing to 1; NULL = 1/B each, Monte Carlo samples).
 * With Ebar = sum_b w_b E_b, F = sum_b w_b O_b (E_b - Ebar) and
 * S = sum_b w_b O_b O_b^T - Obar Obar^T (Obar = sum_b w_b O_b), the system (S + shift I) x = F
 * is solved by conjugate gradients (at most max_iter iterations, until |r| <= tol |F|) and
 * delta = -eta x is written (device float64 [P]); the caller adds it to the parameters and calls
 * dn_model_set_params. energy (device float64 [1], nullable) receives Ebar; iters (host,
 * nullable) the iterations taken. Every sum is float64; S is never formed (each iteration reads
 * O twice). Synchronises the stream every 8 iterations. A complex_out model (complex psi, real
 * parameters) takes O as dn_grad_logpsi writes it, [2][B][P], eloc [B][2] complex, and uses
 * F = Re sum_b w_b conj(O_b - Obar)(E_b - Ebar), S = Re sum_b w_b conj(O_b - Obar)(O_b - Obar)^T;
 * energy is then [2] (re, im). */
dn_status dn_sr_update(dn_model* m, const void* O, const double* eloc, const double* weights, int32_t B,
                       double shift, double eta, int32_t max_iter, double tol, double* delta,
                       double* energy, int32_t* iters, void* stream);

/* dn_logpsi for callers that cannot allocate device memory: code under HIP graph capture,
 * tight sampling or serving loops, harnesses that forbid hipMalloc. The same values as
 * dn_logpsi (the same kernels), but every buffer beyond the caller's inputs and outputs --
 * the forward's fields, its work list and read-out sums -- lives in one file-scope device
 * array of 32 MiB (each GPU the library runs on holds its own copy until the process ends);
 * the call allocates and frees nothing. B is processed in chunks that fit the array; a
 * shape whose single configuration needs more than the array holds gets DN_EUNSUPPORTED
 * (none the library supports does: at most 1.3 MiB). The array keeps the last call's
 * contents, and calls that overlap on one GPU (several streams or host threads) race on
 * it: serialise them. No profiling events are recorded. */
dn_status dn_logpsi_noalloc(dn_model* m, const int8_t* spins, int32_t B, double* logpsi, void* stream);

/* Connected configurations, matrix elements and diagonal energies of H for B samples.
 * M_max must be >= N (Ising) or >= 2N (J1-J2). Outputs: sites [B,M_max,2] (unused rows
 * set to -1), helem [B,M_max] (0 beyond n_conn), n_conn [B], hdiag [B]. */
dn_status dn_connected(const dn_ham_desc* ham, const int8_t* spins, int32_t B, int32_t N,
                       int32_t M_max, int32_t* sites, double* helem, int32_t* n_conn,
                       double* hdiag, void* stream);

/* log psi(s'_m)/psi(s) for every listed element, by DN_PATH_ABACUS (background caches,
 * output links and the slice recurrence; clusters must be one site or two sites at
 * distance <= 2, else DN_EUNSUPPORTED) or DN_PATH_FULL (each s' evaluated from scratch).
 * ABACUS cost per element: networks of one or two blocks do slice-sized work only (the
 * per-sample links -- output links of every block and, for two blocks, block 2's pivot-0
 * link from a frequency-domain composite correlation, App. "Efficient construction of
 * link tensors" -- are built once per sample); deeper networks also propagate each
 * element's change through the frozen blocks 1 .. L-1 over the whole chain (exact,
 * O(N d^2) per element). With inject_phi = 1 the input change of block l + 1 also holds the
 * phi-stream change on S_(l+1), so every depth from two blocks up takes the whole-chain
 * propagation (one block: the slice work only).
 * logpsi (nullable) receives log psi(s); logratio [B, M_max] gets 0 beyond n_conn.
 * n_conn and sites are validated on the device (DN_EINVAL for n_conn outside [0, M_max],
 * a site outside [0, N) or a pair repeating a site); the per-sample work list comes back to
 * the host, so the call synchronises the stream once before its main launches. */
dn_status dn_logratio(dn_model* m, int32_t path, const int8_t* spins, int32_t B,
                      const int32_t* sites, const int32_t* n_conn, int32_t M_max,
                      double* logpsi, double* logratio, void* stream);

/* E_loc = hdiag + sum_{m < n_conn} helem_m exp(logratio_m) (Eq. (local-estimator)). */
dn_status dn_local_energy(const double* hdiag, const double* helem, const int32_t* n_conn,
                          const double* logratio, int32_t B, int32_t M_max, double* eloc,
                          void* stream);

/* dn_local_energy for complex log-ratios (a complex_out model): logratio [B, M_max][2] and
 * eloc [B][2] hold (re, im) pairs; E_loc = hdiag + sum_m helem_m exp(logratio_m). */
dn_status dn_local_energy_complex(const double* hdiag, const double* helem, const int32_t* n_conn,
                                  const double* logratio, int32_t B, int32_t M_max, double* eloc,
                                  void* stream);

/* Whole local estimator: connected elements, log-ratios by `path`, E_loc. logpsi [B]
 * and eloc [B] are required; logratio [B, M_max] may be NULL (then the library keeps it
 * in its workspace). */
dn_status dn_eloc(dn_model* m, int32_t path, const dn_ham_desc* ham, const int8_t* spins,
                  int32_t B, int32_t M_max, double* logpsi, double* logratio, double* eloc,
                  void* stream);

/* Per-sample log-derivatives O[b][p] = d log psi(s_b) / d theta_p for every raw parameter,
 * the quantities variational Monte Carlo with stochastic reconfiguration consumes (Sec. VI).
 * Hand-written reverse mode: a forward pass keeps layer-boundary checkpoints, each block is
 * recomputed from its checkpoint while the adjoints flow back; the S4 parameters follow through
 * the Jacobian of the Green's-function taps (float64, shared by all samples, rebuilt after each
 * dn_model_set_params). grads: [B][P] in the model's field type (float for DN_PREC_FP32, double
 * for DN_PREC_FP64), nullable (then kept in the workspace); logpsi [B] nullable; weights [B] and
 * wsum [P] (float64, both or neither): wsum = sum_b weights[b] O[b][.]. Open and periodic
 * chains (periodic: the Jacobian of the aliased kernel, Sec. V); with inject_phi = 1 the
 * checkpoints hold the mixer inputs h + phi and the phi stream also receives the mixer input's
 * adjoint. A complex_out model has complex O = d Re log psi + i d Im log psi
 * (the parameters are real): grads is then [2][B][P] (all real parts, then all imaginary
 * parts; two reverse passes), wsum [2][P] likewise, logpsi [B][2]. Asynchronous on the stream. */
dn_status dn_grad_logpsi(dn_model* m, const int8_t* spins, int32_t B, double* logpsi, void* grads,
                         const double* weights, double* wsum, void* stream);

/* Launch-shape autotuner: times the ABACUS estimator (dn_eloc) of this model on B_probe
 * synthetic configurations (spins from an integer hash, generated on the device) for each
 * candidate launch shape and keeps the fastest for every later call on the model: the
 * number of 16-site output tiles per wave of the Toeplitz kernel (1..4) and the size of the
 * ABACUS flip chunks (256 MiB, 1 GiB or 3 GiB of flip fields; smaller chunks can stay in
 * the last-level cache, larger ones launch fewer, wider grids). The search is coordinate-wise
 * (tiles first, then chunk size). conv_nt_out and flip_budget_out (nullable) receive the
 * choice. Synchronises the stream; grows the workspace as the candidates need. The Ising
 * model's M_max is N, the J1-J2 chain's 2N. Supports what dn_eloc's ABACUS path supports. */
dn_status dn_autotune(dn_model* m, const dn_ham_desc* ham, int32_t B_probe, int32_t* conv_nt_out,
                      int64_t* flip_budget_out, void* stream);

/* Set the launch shapes dn_autotune would choose, by hand: conv_nt 16-site output tiles per
 * wave of the Toeplitz kernel (0 = by chain length; else 1..4 with the chain length rounded
 * up to 64 a multiple of 16 conv_nt, DN_EINVAL otherwise) and flip_budget bytes of flip
 * fields per ABACUS chunk (0 = 3 GiB). Marks the model as tuned. */
dn_status dn_set_launch_shapes(dn_model* m, int32_t conv_nt, int64_t flip_budget);

/* Arithmetic of the float matrix-core products of the estimator: the Green's-function
 * (Toeplitz mixer) products y_c(i) = sum_k g_c(i - k) x_c(k) (Sec. II, the S4 mixer as a
 * Toeplitz matrix) and the ABACUS deep blocks' channel mixing V and U (Sec. III).
 * DN_PRODUCT_SPLIT3 (the default): each float operand is split into three bfloat16 terms,
 * x = x0 + x1 + x2 exactly (each term the next 8 significant bits), and the six partial
 * products x_a y_b with a + b <= 2 run on the bf16 matrix cores with float32 accumulation;
 * the dropped ones are below 2^-24 |x y|, so the result has the error bound of a float32
 * dot product. DN_PRODUCT_FP32: the float32 matrix cores (one product per term).
 * Float32 models use the setting for both kinds of product; BF16-mixed models take hi + lo
 * bf16 terms (three partial products) where the float models take three terms, for both kinds,
 * and DN_PRODUCT_FP32 moves their Toeplitz products to the float32 matrix cores; float64 models
 * ignore it;
 * the forward and adjoint background passes and the gradients stay on float32 matrix cores.
 * DN_EINVAL for another value. Takes effect on the next call. */
typedef enum { DN_PRODUCT_SPLIT3 = 0, DN_PRODUCT_FP32 = 1 } dn_product_mode;
dn_status dn_set_product_mode(dn_model* m, int32_t mode);

/* Execution modes of dn_ragged_eloc. */
typedef enum {
  DN_RAGGED_EAGER = 0, /* launch every instance's kernels on each call */
  DN_RAGGED_GRAPH = 1  /* record the whole submission once as a HIP graph, then replay it */
} dn_ragged_mode;

/* Local estimator over a ragged batch: n_inst instances, each its own model (shape, width
 * and depth may all differ) with its own Hamiltonian and B[i] samples, in one submission
 * (the estimator of Eq. (local-estimator) through the ABACUS update of Alg. 1 per instance).
 * Host arrays of length n_inst: models (distinct, parameters set, each ABACUS-capable),
 * hams, spins (device [B_i][N_i] int8), B, logpsi (device [B_i] float64; the array or an
 * entry may be NULL), eloc (device [B_i] float64). M_max is N_i (Ising) or 2 N_i (J1-J2).
 * Instances are spread over n_streams (1..8; 0 = 4) HIP streams, heaviest first onto the
 * least-loaded stream. In DN_RAGGED_GRAPH mode the first call with a given set of models,
 * Hamiltonians, sizes and pointers runs eagerly, one instance after another, times each
 * instance, checks every error word (synchronising), and records the submission as one
 * graph with the measured times as costs (models not yet tuned are first passed through
 * dn_autotune on up to 256 of their own samples' shapes); later calls with the same arguments replay it
 * with one graph launch (the spins' values may change; the generator, work lists and
 * counts are rebuilt on the device at each replay). A model used elsewhere in between whose
 * workspace had to grow gets a new recording. Parameter updates (dn_model_set_params) act
 * in place and need no new recording. Replays do not synchronise: a cluster error cannot
 * arise there, since the instances' own generator lists the clusters. The library owns the
 * graphs and streams; dn_model_destroy drops the graphs that use the model. Calls from
 * several host threads are serialised. */
dn_status dn_ragged_eloc(int32_t n_inst, dn_model* const* models, const dn_ham_desc* hams,
                         const int8_t* const* spins, const int32_t* B, double* const* logpsi,
                         double* const* eloc, int32_t n_streams, int32_t mode, void* stream);

/* Kernel classes of the per-launch profile. */
typedef enum {
  DN_K_S4GEN = 0,    /* S4 taps (float64) */
  DN_K_PREP = 1,     /* parameter tables */
  DN_K_PHI = 2,      /* phi stream + vertex of one block */
  DN_K_CONV = 3,     /* Green's-function mixer (Toeplitz product on the matrix cores) */
  DN_K_MIX_FWD = 4,  /* vertex + channel mixing + read-out, forward */
  DN_K_MIX_TAU = 5,  /* adjoint of the last block's vertex (ABACUS output link) */
  DN_K_MIX_DEEP = 6, /* background propagation of the flips' perturbations (ABACUS) */
  DN_K_SLICE = 7,    /* slice recompute of phi / vertices (ABACUS) */
  DN_K_TAIL = 8,     /* per-flip finish: last block's slice + float64 log-ratio (ABACUS) */
  DN_K_GEN = 9,      /* Hamiltonian connected elements */
  DN_K_ELOC = 10,    /* local energy */
  DN_K_OTHER = 11,   /* planning, fills, read-out finalisation */
  DN_K_LINK = 12,    /* block 2's pivot-0 link per sample: transforms + frequency contraction (ABACUS, L = 2) */
  DN_K_COUNT = 13
} dn_kernel_kind;

/* Per-launch profile of a model's kernels. While enabled, every launch the model makes is
 * bracketed by HIP events on its own stream, and its algorithmic work is recorded: flops
 * of the operation as defined (a Toeplitz mixer of n sites counts 2 n^2 per channel, a
 * d x d channel mix 2 d^2 per site) and bytes of its unavoidable HBM traffic (fields read
 * and written once). dn_profile_enable(m, 1) clears the counters; (m, 0) stops recording.
 * dn_profile_read synchronises the device and returns the totals of one kernel class. */
dn_status dn_profile_enable(dn_model* m, int enable);
dn_status dn_profile_read(dn_model* m, int32_t kind, double* total_ms, int64_t* launches,
                          double* flops, double* bytes);

/* Thread-local text of the last error (never NULL). */
const char* dn_last_error(void);

/* Release the model and its device memory (NULL is ignored). */
void dn_model_destroy(dn_model* m);

#ifdef __cplusplus
}
#endif
#endif /* DYSONNET_H */
