/*
 * vqe.h -- C ABI of the MI355X (gfx950) VQE hot-path library, libvqe.so.
 *
 * The calls follow the statement of the problem in arXiv 2601.09951:
 *   prepare the reference state        (Section 3.3, Eq. 4: |HF>)
 *   apply the ansatz U(theta)          (Section 3.3, Eqs. 4-5; Section 4.3)
 *   expect <psi|H|psi> of a Pauli sum  (Section 3.1, Eq. 2; Section 3.2)
 *   gradient dE/dtheta                 (Algorithm 1; Sections 4.3, 5.2.5)
 *   optimiser step                     (Section 3.4, Adam, lr 0.01)
 *   the per-bond-length loop           (Algorithm 1, Section 4.2; Eq. 7)
 *
 * Conventions (shared by every call)
 * ----------------------------------
 * - A state on n qubits is complex128 [batch][2^n], re/im interleaved,
 *   row-major, in device memory.  Wire w is bit (n-1-w) of the amplitude
 *   index: a printed ket |w0 w1 ... w_{n-1}> reads as the binary expansion
 *   of its index (|1100> is index 12 at n = 4).
 * - A Pauli string is (xmask, zmask) over amplitude-index bits: bit b of
 *   xmask is set for X or Y on the wire owning bit b, bit b of zmask for Z
 *   or Y; the string acts as P|b> = i^{popcount(x&z)} (-1)^{popcount(z&b)}
 *   |b xor x>.
 * - Parameters are float64 [batch][n_params]; energies float64 [batch];
 *   gradients float64 [batch][n_params]; all in device memory.
 * - `stream` is a hipStream_t (NULL = the null stream).  Every call that
 *   takes a stream only enqueues work on it and returns; results are valid
 *   once the stream has reached that point.
 * - Memory passed in is borrowed: the library never frees caller memory and
 *   never keeps a pointer to it after the call returns.  Handles own the
 *   device tables they allocate, until destroyed.
 * - Every call returns VQE_OK (0) or a negative error code; no C++
 *   exception crosses this boundary.  On error nothing is enqueued, and
 *   vqe_last_error(ctx) describes the cause.
 * - A context is bound to one device.  Calls on one context must not run
 *   concurrently from several host threads.
 */
#ifndef VQE_H
#define VQE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------- */
#define VQE_OK 0
#define VQE_EINVAL (-1)       /* bad argument: null pointer, size, wire, NaN/Inf */
#define VQE_ENOMEM (-2)       /* device memory or the context's budget exhausted */
#define VQE_EUNSUPPORTED (-3) /* n outside [1, VQE_MAX_QUBITS], unknown gate kind */
#define VQE_EHIP (-4)         /* a HIP runtime call failed; message in the context */

#define VQE_MAX_QUBITS 34

/* ---- gate kinds (Section 3.3 and the hardware-efficient ansatz) --------
 * Rotations are U(a) = exp(-i a G / 2) with generator G:
 *   RX: G = X; RY: G = Y; RZ: G = Z;
 *   SINGLE_EXC (wires a, b): |01> -> c|01> + s|10>, |10> -> c|10> - s|01>,
 *       c = cos(a/2), s = sin(a/2), G = (Y(x)X - X(x)Y) / 2;
 *   DOUBLE_EXC (wires a, b, c, d): |0011> -> c|0011> + s|1100>,
 *       |1100> -> c|1100> - s|0011>, identity elsewhere: the Givens-rotation
 *       reading of Eq. (5) (whose printed exponent is not anti-Hermitian).
 * Fixed gates: H, X, CNOT (control = first wire), CZ. */
enum {
    VQE_GATE_RX = 0,
    VQE_GATE_RY = 1,
    VQE_GATE_RZ = 2,
    VQE_GATE_H = 3,
    VQE_GATE_X = 4,
    VQE_GATE_CNOT = 5,
    VQE_GATE_CZ = 6,
    VQE_GATE_SINGLE_EXC = 7,
    VQE_GATE_DOUBLE_EXC = 8
};

/* optimisers for vqe_run */
enum { VQE_OPT_ADAM = 0, VQE_OPT_GD = 1 };

typedef struct vqe_ctx *vqe_ctx_t;
typedef struct vqe_ham *vqe_ham_t;
typedef struct vqe_circ *vqe_circ_t;

/* ---- context ----------------------------------------------------------- */

/* Create a context on HIP device `device` (made current for every later
 * call on this context).  *out receives the handle.  device = -1 creates a
 * host-only planning context: Hamiltonians, circuits, workspace sizes and
 * schedule exports work without a GPU; calls that enqueue device work fail
 * with VQE_EUNSUPPORTED.  Errors: EINVAL (out NULL, bad device), EHIP. */
int vqe_ctx_create(int device, vqe_ctx_t *out);

/* Destroy a context and everything it caches.  Handles created from it must
 * be destroyed first.  Waits for nothing: the caller synchronises. */
int vqe_ctx_destroy(vqe_ctx_t ctx);

/* Cap on the device memory the context may allocate for its own tables and
 * caches (0 = no cap).  Allocations that would exceed it fail with ENOMEM. */
int vqe_ctx_set_mem_budget(vqe_ctx_t ctx, size_t bytes);

/* Tile geometry of the state passes: k_fwd / k_rev = log2 of the number of
 * amplitudes a workgroup holds in LDS in forward / reverse (adjoint) passes
 * (forward 6..13, reverse 6..12), c_low = number of lowest index bits every
 * tile contains (contiguous runs of 2^c_low amplitudes); c_low >= 2 and
 * k - c_low >= 4 for both k, so a four-wire gate always fits a tile.
 * Defaults: k_fwd 12, k_rev 11, c_low 3 (runs of one 128-byte line).  Pass 0
 * to keep a value.  Changes apply to plans built afterwards.  A flip group
 * whose X/Y bits outside the lowest c_low bits number more than k - c_low
 * fits no tile; it is evaluated by a whole-state pair sweep of its own (one
 * more read of the state per such group). */
int vqe_ctx_set_tile(vqe_ctx_t ctx, int k_fwd, int k_rev, int c_low);

/* How vqe_run executes: mode 0 (default) runs the whole loop in one
 * persistent launch per batch when a state fits one workgroup's LDS (n up to
 * 10 with the default tiles), else per-step launches; mode 1 always uses
 * per-step launches (one energy_grad sequence and one optimiser launch per
 * step). */
int vqe_ctx_set_loop_mode(vqe_ctx_t ctx, int mode);

/* Kernel variant of the state passes: staged = 2 (default) runs forward and
 * adjoint passes made of uncontrolled one-qubit gates, X and CNOT as fused
 * stages (one 2x2 per qubit, the CNOT / X network folded into data
 * movement; in adjoint passes the gradient terms of a qubit's gates come
 * from three pair sums of the states before them) and everything else as
 * staged = 1; staged = 1 applies the gates of a pass in register stages of
 * four (forward) or three (adjoint) tile bits (tiles of 8 or more bits);
 * staged = 0 applies one gate per LDS round trip and also accumulates
 * H psi by pair updates in LDS, where staged >= 1 gathers every amplitude
 * of H psi in registers (tiles of 8 to 11 bits).  All compute the same
 * result up to rounding; the switch exists for measurement. */
int vqe_ctx_set_staged(vqe_ctx_t ctx, int staged);

/* Launch graphs (on = 1; off by default): a launch sequence of vqe_energy,
 * vqe_energy_grad or one optimiser step of vqe_run's per-step loop that is
 * seen a second time with identical arguments (pointers included) is
 * captured into a hipGraph, which is launched instead of the individual
 * kernels from then on; the optimiser step reads its step index from the
 * workspace, so every step of a loop is the same graph.  The second call
 * waits once for its stream and for pending table uploads before capturing.
 * A graph is dropped when a Pauli plan it reads is retired (a Hamiltonian
 * destroyed, the plan cache flushed) or its circuit is destroyed.  Kernel
 * timing (vqe_ctx_set_profiling) keeps calls eager.  on = 0 drops every
 * graph.  Off by default: on the measured workloads (4 to 26 qubits) replays
 * were no faster than eager launches, and for a call of a few short kernels
 * a graph launch costs more host time than the launches it replaces; it is
 * for callers whose host loop cannot keep the GPU busy. */
int vqe_ctx_set_graphs(vqe_ctx_t ctx, int on);

/* Graphs captured and launched so far, and graphs cached now (any pointer
 * may be NULL). */
int vqe_ctx_graph_stats(vqe_ctx_t ctx, int64_t *captures, int64_t *launches, int64_t *cached);

/* ---- autotuning ----------------------------------------------------------
 * vqe_autotune times vqe_energy (want_grad = 0) or vqe_energy_grad
 * (want_grad = 1) on the caller's arguments for candidate execution choices
 * and keeps the fastest for (circuit, batch, want_grad); later calls of
 * vqe_energy / vqe_energy_grad / vqe_workspace_bytes with that circuit and
 * batch (and vqe_run's per-step loop, with the energy + gradient choice) use
 * it instead of the context defaults.  Candidates, one coordinate at a time
 * from the defaults (coordinate descent, a change kept when it is 2 % faster):
 * forward tile bits k_fwd 8..min(n, 13), adjoint tile bits k_rev 8..min(n,
 * 12), contiguous low bits c_low 2..4, the batch tile (instances per launch
 * sequence: batch / 2, batch / 4, ..., 1; a batch then runs as consecutive
 * chunks, so that a chunk's states can stay in the last-level cache), and
 * the cap on workgroups per instance (256, 1024, 4096; the default cap is
 * 8192, and a pass uses about one workgroup per four tiles, at least 512,
 * within the cap).  Each candidate runs
 * twice untimed (plans, uploads, graph capture) and then at least 3 times
 * (until 20 ms) between HIP events on `stream`, with outputs and a workspace
 * that the tuner allocates for each candidate's size (set-up work: size the
 * caller's workspace with vqe_workspace_bytes after tuning); a candidate that
 * cannot evaluate the Hamiltonian with its tiles is skipped.  States of at
 * most 8 qubits are one tile at every width: only the defaults are timed.
 * The host waits for the stream.  Errors: EINVAL, ENOMEM (the defaults could
 * not be evaluated), EHIP. */
typedef struct {
    int k_fwd, k_rev, c_low, wg_max;
    int64_t batch_tile;  /* instances per launch sequence */
    double ms_default;   /* ms per call with the context defaults */
    double ms_tuned;     /* ms per call with the chosen configuration */
    int candidates;      /* configurations timed */
} vqe_tune_result;

int vqe_autotune(vqe_ctx_t ctx, vqe_circ_t circ, int n_hams, const vqe_ham_t *hams, int64_t batch,
                 uint64_t ref_index, int want_grad, const double *theta, void *stream, vqe_tune_result *out);

/* Use `cfg` (its k_fwd, k_rev, c_low, wg_max and batch_tile; the timing
 * fields are ignored) for (circuit, batch, want_grad) as if vqe_autotune had
 * chosen it: a configuration found earlier can be reused without timing.
 * Errors: EINVAL (ranges as vqe_ctx_set_tile, wg_max >= 1, batch_tile >= 1). */
int vqe_tune_set(vqe_ctx_t ctx, vqe_circ_t circ, int64_t batch, int want_grad, const vqe_tune_result *cfg);

/* Forget every tuned choice of the context (calls use the defaults again). */
int vqe_ctx_clear_tuning(vqe_ctx_t ctx);

/* Reserve `bytes` of context scratch now (used by vqe_expect and
 * vqe_apply_ansatz for per-launch tables), so later calls do not allocate. */
int vqe_ctx_reserve(vqe_ctx_t ctx, size_t bytes);

/* ---- kernel timing (measurement) ----------------------------------------
 * With profiling on, the library brackets each launch of the state passes,
 * the Pauli sweeps and the persistent loop with a pair of HIP events on the
 * launch's own stream and accumulates, per kernel (and role), the launch
 * count, the summed event durations and the algorithmic HBM bytes of those
 * launches (every amplitude read and written once per forward pass: 32 B;
 * adjoint pass with psi and lambda: 64 B; expectation sweep: 16 B; H psi
 * sweep: 32 B for the first, 48 B for later sweeps; times 2^n per state and
 * the batch).  The events add a few microseconds per launch; launches on a
 * stream that is being captured are not timed. */
typedef struct {
    char name[48];      /* kernel and role, NUL-terminated */
    int64_t launches;
    double total_ms;    /* summed event-measured durations */
    double bytes;       /* algorithmic HBM bytes of those launches (0: not counted) */
} vqe_kernel_stat;

/* on = 1 starts timing launches made afterwards, 0 stops. */
int vqe_ctx_set_profiling(vqe_ctx_t ctx, int on);

/* Wait for every timed launch, then copy up to `capacity` per-kernel totals
 * into out (sorted by name) and the number of kernels into *count (which may
 * exceed capacity).  reset = 1 clears the totals afterwards.  out may be NULL
 * when capacity is 0. */
int vqe_ctx_profile(vqe_ctx_t ctx, vqe_kernel_stat *out, int capacity, int *count, int reset);

/* ---- streams for concurrent callers ------------------------------------
 * A HIP stream (default priority, every compute unit) on a hardware queue of
 * its own.  The runtime maps ordinary streams onto a small pool of hardware
 * queues, and the work of streams that share a queue runs in submission
 * order; a serving loop that lets short requests pass a long batch therefore
 * runs each request class on such a stream.  *stream receives a hipStream_t
 * owned by the caller until vqe_stream_destroy (which does not wait for the
 * stream's work).  Errors: EINVAL (NULL out), EUNSUPPORTED (host-only
 * context), EHIP. */
int vqe_stream_create(vqe_ctx_t ctx, void **stream);
int vqe_stream_destroy(vqe_ctx_t ctx, void *stream);

/* Text of the last error on this context (never NULL). */
const char *vqe_last_error(vqe_ctx_t ctx);

/* Name of an error code (never NULL). */
const char *vqe_strerror(int code);

/* ---- Hamiltonians (Section 3.2, Eq. 3 and its Jordan-Wigner image) ----- */

/* A Pauli sum H = sum_t coeff[t] P(xmask[t], zmask[t]) on n_qubits qubits.
 * Host arrays of length n_terms are copied; equal strings are merged; the
 * identity string (x = z = 0) is allowed.  Errors: EINVAL (NaN/Inf
 * coefficient, mask bits at or above n_qubits, n_terms < 1),
 * EUNSUPPORTED (n_qubits outside [1, VQE_MAX_QUBITS]), ENOMEM, EHIP. */
int vqe_ham_create(vqe_ctx_t ctx, int n_qubits, int64_t n_terms, const uint64_t *xmask,
                   const uint64_t *zmask, const double *coeff, vqe_ham_t *out);

/* The qubit Hamiltonian of Eq. (3) from spatial-orbital integrals, mapped by
 * Jordan-Wigner on n_qubits = 2 * n_orb interleaved spin orbitals (wire 2p =
 * orbital p spin alpha, 2p+1 = spin beta; |1> = occupied):
 *   H = e_core + sum_{PQ} h_PQ a+_P a_Q + 1/2 sum_{PQRS} (ps|qr) a+_P a+_Q a_R a_S
 * with spin conserved on each one-body and two-body vertex.  h1 is the host
 * array [n_orb][n_orb], h2 the host array [n_orb]^4 of chemist-notation
 * integrals (pq|rs); both are read, not kept.  Coefficients with magnitude
 * <= 1e-14 are dropped.  Errors: EINVAL (NaN/Inf, a complex coefficient
 * from non-symmetric input), EUNSUPPORTED (n_orb < 1 or 2*n_orb > 34). */
int vqe_ham_from_integrals(vqe_ctx_t ctx, int n_orb, const double *h1, const double *h2,
                           double e_core, vqe_ham_t *out);

/* Sizes of a Hamiltonian: qubits, merged terms, distinct flip masks. */
int vqe_ham_info(vqe_ham_t ham, int *n_qubits, int64_t *n_terms, int64_t *n_groups);

/* Copy the merged terms (sorted by (xmask, zmask)) into host arrays of
 * length n_terms as reported by vqe_ham_info. */
int vqe_ham_terms(vqe_ham_t ham, uint64_t *xmask, uint64_t *zmask, double *coeff);

int vqe_ham_destroy(vqe_ham_t ham);

/* ---- Hamiltonian families (Eq. 3 for many integral sets, on the device) --
 * The Jordan-Wigner coefficients of Eq. (3) are linear in the integrals.  A
 * family holds that linear map for n_orb spatial orbitals (built once on the
 * host) and device storage for the coefficients of `capacity` members; the
 * coefficients of any set of members are then computed on the device from
 * integrals already in device memory (one sparse product per member, no
 * host round trip), which is how a potential-energy scan builds H(d_i) for
 * every bond length.  Integrals must be symmetric (h1 symmetric, h2 with the
 * 8-fold permutational symmetry); the map reads one entry per symmetry
 * class. */
typedef struct vqe_hfam *vqe_hfam_t;

int vqe_hfam_create(vqe_ctx_t ctx, int n_orb, int64_t capacity, vqe_hfam_t *out);

/* qubits (2 n_orb), Pauli strings of the map, integral inputs per member
 * (1 + n_orb^2 + n_orb^4, laid out {e_core, h1[n_orb][n_orb], h2[n_orb]^4}). */
int vqe_hfam_info(vqe_hfam_t fam, int *n_qubits, int64_t *n_terms, int64_t *n_inputs);

/* A Hamiltonian handle for member `index` (0 <= index < capacity): its strings
 * are the family's, its coefficients the member's device row.  Usable
 * wherever a vqe_ham_t is taken; all Hamiltonians of one call must come from
 * one family or from none.  Destroy members before their family. */
int vqe_hfam_member(vqe_hfam_t fam, int64_t index, vqe_ham_t *out);

/* Coefficients of members [first, first + count) from device integrals
 * float64 [count][n_inputs]; enqueued on `stream`.  Calls on the same stream
 * that evaluate these members see the new coefficients. */
int vqe_hfam_set_integrals(vqe_ctx_t ctx, vqe_hfam_t fam, int64_t first, int64_t count,
                           const double *integrals, void *stream);

int vqe_hfam_destroy(vqe_hfam_t fam);

/* ---- circuits (the ansatz U(theta) of Eq. 4) --------------------------- */

/* A gate list applied in order.  kind[g] is a VQE_GATE_* code; wires is the
 * host array [n_gates][4] listing gate g's wires in the order its
 * definition uses (unused slots -1); param_idx[g] indexes the parameter
 * vector (-1 = fixed gate with angle fixed_angle[g]; fixed_angle may be NULL
 * when no gate is fixed-angle); n_params is the parameter-vector length.
 * Host arrays are copied.  Errors: EINVAL (wire out of range or repeated,
 * param_idx >= n_params, parameter on a non-rotation gate), EUNSUPPORTED
 * (unknown kind, n_qubits out of range). */
int vqe_circ_create(vqe_ctx_t ctx, int n_qubits, int64_t n_gates, const int32_t *kind,
                    const int32_t *wires, const int32_t *param_idx, const double *fixed_angle,
                    int32_t n_params, vqe_circ_t *out);

int vqe_circ_destroy(vqe_circ_t circ);

/* ---- workspace --------------------------------------------------------- */

/* Bytes of device workspace that vqe_energy (want_grad = 0),
 * vqe_energy_grad (want_grad = 1), vqe_run (want_grad = 2) or
 * vqe_grad_shift (want_grad = 3) needs for `batch` instances: the state, the
 * adjoint state lambda = H psi, and small per-launch tables; for vqe_run on
 * states of at most 8 qubits also the persistent loop's history of the
 * state on every gate's pairs, (gates + 1) * 4 KB per instance at 8 qubits
 * (2 KB below).  A state is batch * 2^n * 16 bytes. */
int vqe_workspace_bytes(vqe_ctx_t ctx, vqe_circ_t circ, int n_hams, const vqe_ham_t *hams,
                        int64_t batch, int want_grad, size_t *bytes);

/* ---- the hot path ------------------------------------------------------ */

/* psi[b] <- e_ref for every instance b (Eq. 4's |HF>, or |0...0>).
 * psi: device complex128 [batch][2^n_qubits]. */
int vqe_prepare_reference(vqe_ctx_t ctx, int n_qubits, int64_t batch, uint64_t ref_index,
                          void *psi, void *stream);

/* psi[b] <- U(theta[b]) psi[b] in place, gates in list order.  theta: device
 * float64 [batch][n_params]. */
int vqe_apply_ansatz(vqe_ctx_t ctx, vqe_circ_t circ, int64_t batch, const double *theta,
                     void *psi, void *stream);

/* vqe_apply_ansatz for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and result, but the per-call gate and fused-stage
 * matrices (batch * (gates + fused slots) * 64 bytes) go to a static device
 * array of VQE_NOALLOC_SCRATCH_BYTES per GPU instead of context scratch, and
 * the call makes no device or host allocation.  The circuit's forward plan
 * for the context's current tiles must exist: vqe_circ_create builds it, and
 * any evaluation of the circuit after vqe_ctx_set_tile rebuilds it.  Every
 * call on one GPU uses that GPU's single array, so calls that overlap on one
 * GPU (other streams, other contexts, other threads) race; serialise them.
 * Errors: as vqe_apply_ansatz; EINVAL when the matrices exceed the array
 * (the message gives the largest batch) or the plan is missing. */
#define VQE_NOALLOC_SCRATCH_BYTES (8u << 20)
int vqe_apply_ansatz_noalloc(vqe_ctx_t ctx, vqe_circ_t circ, int64_t batch, const double *theta,
                             void *psi, void *stream);

/* energy[b] = <psi[b]|H_b|psi[b]> (real part; Eq. 2).  hams has n_hams = 1
 * (shared) or n_hams = batch entries, all on the state's qubit count.  Terms
 * are evaluated grouped by flip mask, one tile sweep serving every group
 * whose flip bits the tile holds.  energy: device float64 [batch]. */
int vqe_expect(vqe_ctx_t ctx, int n_hams, const vqe_ham_t *hams, int64_t batch, const void *psi,
               double *energy, void *stream);

/* energy[b] = <psi_b|H_b|psi_b> with psi_b = U(theta[b]) e_ref: prepare, apply
 * and expect in one call, using caller workspace (at least
 * vqe_workspace_bytes(..., want_grad = 0)) instead of context scratch.
 * energy: device float64 [batch]. */
int vqe_energy(vqe_ctx_t ctx, vqe_circ_t circ, int n_hams, const vqe_ham_t *hams, int64_t batch,
               uint64_t ref_index, const double *theta, double *energy, void *workspace,
               size_t ws_bytes, void *stream);

/* out[b] = H_b psi[b] (the adjoint seed lambda).  out must not alias psi. */
int vqe_apply_hamiltonian(vqe_ctx_t ctx, int n_hams, const vqe_ham_t *hams, int64_t batch,
                          const void *psi, void *out, void *stream);

/* Energy and adjoint gradient for every instance: prepare e_ref, apply
 * U(theta[b]), lambda = H psi with E fused, then the reverse sweep
 *   g_l = Im <lambda_l|G_l|psi_l>,  psi <- U_l^dag psi,  lambda <- U_l^dag lambda
 * accumulated per parameter (dE/dtheta_p = sum of g_l over gates using p).
 * energy: device [batch]; grad: device [batch][n_params]; workspace: device
 * memory of at least vqe_workspace_bytes(..., want_grad = 1). */
int vqe_energy_grad(vqe_ctx_t ctx, vqe_circ_t circ, int n_hams, const vqe_ham_t *hams,
                    int64_t batch, uint64_t ref_index, const double *theta, double *energy,
                    double *grad, void *workspace, size_t ws_bytes, void *stream);

/* Energy and the parameter-shift gradient of Algorithm 1 (Section 4.3: two
 * evaluations per parameter): every instance is expanded into shifted rows,
 * gate by gate, evaluated as one batch of states (prepare, apply, expect),
 * and combined per parameter (the chain rule sums shared parameters):
 *   RX, RY, RZ (generator eigenvalues +-1):  [E(a + pi/2) - E(a - pi/2)] / 2
 *   SINGLE_EXC, DOUBLE_EXC (eigenvalues -1, 0, 1):
 *     d+ [E(a + pi/2) - E(a - pi/2)] - d- [E(a + 3pi/2) - E(a - 3pi/2)],
 *     d+- = (sqrt2 +- 1) / (4 sqrt2).
 * Exact for these gates, so it equals the adjoint gradient up to rounding.
 * energy: device [batch]; grad: device [batch][n_params]; workspace: at
 * least vqe_workspace_bytes(..., want_grad = 3).  batch times the rows per
 * instance (1 + 2 per rotation + 4 per excitation) must not exceed 65535. */
int vqe_grad_shift(vqe_ctx_t ctx, vqe_circ_t circ, int n_hams, const vqe_ham_t *hams, int64_t batch,
                   uint64_t ref_index, const double *theta, double *energy, double *grad,
                   void *workspace, size_t ws_bytes, void *stream);

/* One Adam step in place (Section 3.4; Kingma-Ba with epsilon outside the
 * square root): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * theta -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).  t >= 1.
 * All arrays device float64 [batch][n_params]. */
int vqe_adam_step(vqe_ctx_t ctx, int64_t batch, int32_t n_params, double *theta, double *m,
                  double *v, const double *grad, int32_t t, double lr, double b1, double b2,
                  double eps, void *stream);

/* The per-bond-length loop of Algorithm 1 for a batch of independent
 * instances (Eq. 7): theta[b] (device, in: theta_0, out: final) takes
 * `iters` optimiser steps (VQE_OPT_ADAM with lr, b1, b2, eps; or VQE_OPT_GD
 * with step lr), each on the adjoint gradient at the current theta.
 * energies: device float64 [batch][iters + 1]: the energy before each step,
 * then the energy at the final theta.  Small states run the whole loop in
 * one persistent launch (one workgroup per instance; the workspace keeps
 * the state on each gate's pairs after the forward sweep for the reverse
 * sweep, so calls that overlap on one workspace race); larger ones loop over
 * vqe_energy_grad-style launches on the stream.  workspace: at least
 * vqe_workspace_bytes(..., want_grad = 2). */
int vqe_run(vqe_ctx_t ctx, vqe_circ_t circ, int n_hams, const vqe_ham_t *hams, int64_t batch,
            uint64_t ref_index, double *theta, int32_t iters, int32_t optimizer, double lr,
            double b1, double b2, double eps, double *energies, void *workspace, size_t ws_bytes,
            void *stream);

/* ---- schedule inspection (tooling and tests) ---------------------------
 * Copy a compiled schedule into host memory.  If buf is NULL or buf_bytes is
 * smaller than needed, only *needed is written.  Layouts (little endian,
 * natural alignment):
 *
 * vqe_circ_plan_export: int32 {n_passes, n_ops, geom_bytes (72), op_bytes
 *   (48), n_stages, n_stage_ops, stage_bytes (48), stage_op_bytes (48)},
 *   then per pass {geom, int32 op_begin, op_count, n_param_ops,
 *   stage_begin, stage_count, fstage_begin, fstage_count, 0}, then n_ops
 *   op records, n_stages stage records and n_stage_ops stage-op records,
 *   then the fused stages: int32 {n_fstages, fstage_bytes (104), n_fconds,
 *   fcond_bytes (24), n_slots, n_slot_gates, n_phases, phase_bytes (16)},
 *   n_fstages records {uint8 rpos[4], cpos[12], uint16 lr[16], lc[12], c0,
 *   perm, int32 na, cond_begin, cond_count, slot, nb, phase_begin,
 *   phase_count} (apply the fused 2x2 of slot + j to register bit j < na,
 *   then the stage's parity phases, then store register i of sub-cube u at
 *   tile index (xor of lc[j] over the bits j of u) ^ lr[i] ^ c0 ^ (xmask of
 *   every active conditional record) when perm = 1), n_fconds records
 *   {uint64 cmo, cvo, uint32 xmask, 0} (active when (tile base & cmo) ==
 *   cvo), int32 slot offsets [n_slots + 1], the gate of each slot entry and its
 *   int32 info ((parametric gate index + 1) << 4 | class << 2 | generator,
 *   class and generator as in the op record).  Forward
 *   stages multiply a slot's matrices in list order (an empty slot is the
 *   identity); adjoint stages (nb = 3) undo them one by one, and there the
 *   store map is the inverse network of the next gates in reversed order.
 *   Then n_phases records {uint32 mask, cbit, int32 gate, info}: an RZ met
 *   after the network had touched its qubit, applied in the stage's index
 *   frame v as the gate's diagonal entry u00 or u11 chosen by
 *   parity(mask & v) ^ cbit.  geom = int32 {n, k, c,
 *   n - k}, uint8 tpos[16]
 *   (index bit of tile bit i), uint8 opos[40] (index bit of tile-number bit
 *   i).  op = uint32 m, uint32 fixed_bits, uint64 cmask_out, uint64
 *   cval_out, int32 gate, int32 pgate, int16 cls (0 general, 1 diagonal,
 *   2 swap, 3 real general), int16 gen (0 none, 1 X, 2 Y, 3 Z), int8 nfix, uint8
 *   fixpos[7]: the op updates the pairs p0 = (j with zero bits inserted at
 *   fixpos[0..nfix)) | fixed_bits, p1 = p0 ^ m, j < 2^(k - nfix), of the
 *   tiles whose base satisfies (base & cmask_out) == cval_out.  For tiles
 *   of 8 or more bits the same ops are also grouped into register stages:
 *   stage = uint8 rpos[4] (tile bits held in registers), uint8 cpos[12]
 *   (the other tile bits, ascending), int32 op_begin, op_count,
 *   n_param_ops, nbits (register bits: 4 forward, 3 adjoint), uint64 cpos
 *   packed 4 bits apiece, uint32 rpos packed 4 bits apiece, 0; stage op =
 *   uint64 cmo, cvo (controls outside the tile),
 *   uint32 cmt, cvt (tile controls outside the registers), int32 gate,
 *   pgate, uint8 M, lo, cmr, cvr (register flip mask, lower-element
 *   pattern, register controls), uint8 swap, cls, gen, 0, uint16 amask
 *   (bit i set when pair i passes the register predicates), 3 x uint16 0:
 *   register index i pairs with i ^ M (i < 2^nbits) when (i & M) == lo and
 *   the controls hold; swap = 1 means the lower index holds the op's second
 *   element.
 *   reverse = 1 exports the adjoint sweep's schedule (gates in reverse).
 *
 * vqe_ham_plan_export (for_gradient = 0: the expectation schedule, 1: the
 *   H psi schedule): int32 {n_sweeps, n_groups, n_union_groups, n_inst,
 *   n_terms, geom_bytes, group_bytes (16), term_bytes (24)}, per sweep
 *   {geom, int32 group_begin, group_count, 0, 0}, groups {uint32 floc,
 *   uint32 pivot, int32 union_group, 0}, int32 toff[n_inst][n_union][3]
 *   (begin of real-phase terms, begin of imaginary-phase terms, end), terms
 *   {uint64 z, uint32 zloc, 0, double w}, then int32 {n_wide, wide_bytes
 *   (16)} and n_wide records {uint64 f, int32 pivot, int32 union_group}: the
 *   flip groups too wide for a tile, each evaluated over the whole state on
 *   the pairs (b, b ^ f) with bit pivot of b clear (their terms' zloc is 0). */
int vqe_circ_plan_export(vqe_ctx_t ctx, vqe_circ_t circ, int reverse, void *buf, size_t buf_bytes,
                         size_t *needed);
int vqe_ham_plan_export(vqe_ctx_t ctx, int n_hams, const vqe_ham_t *hams, int64_t batch,
                        int for_gradient, void *buf, size_t buf_bytes, size_t *needed);

#ifdef __cplusplus
}
#endif
#endif /* VQE_H */
