/*
 * tq.h -- C ABI of libtq, an MI355X (gfx950) simulator for parameterised quantum circuits.
 *
 * The operations follow the TeD-Q paper (arXiv 2301.05451):
 *   - state-vector mode, Sec. 3.1: |psi> = U |psi_0>, gates applied in program order to a
 *     2^n complex vector, initial state |0..0> or a caller vector of length 2^n;
 *   - the VQC cost of Sec. 4: f = <psi| O |psi> for O a real combination of Pauli-Z strings;
 *   - gradients of f with respect to gate parameters (Sec. 4; the values are those of the
 *     parameter-shift rule of Sec. 4.2, computed here by one reverse adjoint sweep);
 *   - tensor-network mode, Sec. 3.2: a closed network with every index of dimension 2,
 *     contracted pairwise along a binary tree (Sec. 3.2.2), optionally sliced (Sec. 3.2.3);
 *   - the small MLP kernels used by the runtime cost model that ranks contraction trees.
 *
 * Conventions (all entry points):
 *   - Qubit q of an n-qubit register is bit position n-1-q of the amplitude index (qubit 0
 *     is the most significant bit; Sec. 5.1, zeroth qubit on the left).
 *   - States are interleaved complex arrays: float2 (TQ_C64) or double2 (TQ_C128).
 *     Parameters are real arrays of the matching precision (float or double).
 *   - Pointers named d_* are device pointers owned by the caller; the library never frees
 *     or reallocates them. Pointers without the prefix are host pointers, read during the
 *     call only. The context owns its internal device scratch (schedules, gate matrices,
 *     reduction partials).
 *   - Every call is asynchronous on `stream` (a hipStream_t, NULL = default stream) and
 *     validates its arguments on the host before anything is launched. On failure it
 *     returns a non-zero tq_status and tq_last_error() describes the problem; nothing has
 *     been launched. A kernel fault surfaces as TQ_EHIP from a later call.
 *   - A context is bound to one device and is not thread-safe.
 */
#ifndef LIBTQ_TQ_H_
#define LIBTQ_TQ_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TQ_OK = 0,
  TQ_EINVAL = 1,     /* bad argument: op code, qubit index, duplicate qubits, null pointer */
  TQ_ESIZE = 2,      /* size mismatch, e.g. a state that is not 2^n long (Sec. 3.1) */
  TQ_ENOTSUP = 3,    /* valid but unsupported request (e.g. n > 34) */
  TQ_EHIP = 4,       /* a HIP runtime call failed */
  TQ_EWORKSPACE = 5, /* caller workspace smaller than the size query returned */
  TQ_ENOMEM = 6      /* internal device allocation failed */
} tq_status;

typedef enum { TQ_C64 = 0, TQ_C128 = 1 } tq_dtype;

/* Gate codes. Matrices (c = cos(a/2), s = sin(a/2)):
 *   H, X, Y, Z: textbook; RX(a) = [[c,-is],[-is,c]]; RY(a) = [[c,-s],[s,c]] (printed in
 *   Sec. 3.2.1); RZ(a) = diag(e^{-ia/2}, e^{ia/2}); U3(th,ph,la) = [[c,-e^{i la}s],
 *   [e^{i ph}s, e^{i(ph+la)}c]] (c,s of th); ROT(ph,th,om) = RZ(om) RY(th) RZ(ph);
 *   CNOT(control, target) = |0><0| x I + |1><1| x X (the block form of Sec. 3.2.1);
 *   CZ = diag(1,1,1,-1); RZZ(a) = exp(-i a Z Z / 2);
 *   CRX(a), CRY(a), CRZ(a) on (control, target) = |0><0| x I + |1><1| x R(a), the controlled
 *   rotations whose generators have four eigenvalues (Sec. 4.2, four-term shift rule); the
 *   library applies them through exact identities with H, RZ and RZZ (tq_lower_gates). */
enum {
  TQ_H = 0, TQ_X, TQ_Y, TQ_Z, TQ_RX, TQ_RY, TQ_RZ, TQ_U3, TQ_ROT, TQ_CNOT, TQ_CZ, TQ_RZZ,
  TQ_CRX, TQ_CRY, TQ_CRZ,
  TQ_NUM_OPS
};


/* One gate. Angle slot j (j < number of angles of op) is pscale[j] * params[pidx[j]] when
 * pidx[j] >= 0 (index into this circuit's parameter vector), else the constant pscale[j].
 * Unused q / pidx entries should be -1. 48 bytes. */
typedef struct {
  int32_t op;
  int32_t q[2];
  int32_t pidx[3];
  double pscale[3];
} tq_gate;

/* Host only: writes to `out` (capacity `cap` records; may be NULL to query the count) the
 * gate list as the kernels apply it: controlled rotations replaced by H / RZ / RZZ pieces
 * (CRZ(a) = RZ_t(a/2) RZZ(-a/2); CRX(a) = H_t CRZ(a) H_t; CRY(a) = RZ_t(pi/2) CRX(a)
 * RZ_t(-pi/2)), each piece keeping the parameter with its scale halved (so gradients
 * summed over the pieces are the gate's own), other gates copied. Returns the number of
 * gates, or -1 (tq_last_error) on a NULL input with n_in > 0, a negative n_in, or cap too
 * small. */
int32_t tq_lower_gates(const tq_gate* in, int32_t n_in, tq_gate* out, int32_t cap);

/* One term of an observable: coeff * prod_{q: bit q of mask set} Z_q, added to output
 * `obs`. 24 bytes. */
typedef struct {
  uint64_t mask;
  double coeff;
  int32_t obs;
  int32_t _pad;
} tq_zterm;

/* A batch of circuits sharing one gate array, one parameter array and one state array.
 * All member arrays are host arrays of length `count`. Circuit i has n_qubits[i] qubits,
 * gates gates[gate_off[i] .. gate_off[i] + n_gates[i]), parameters
 * d_params[param_off[i] ..] and amplitudes d_states[state_off[i] .. + 2^n_qubits[i]).
 * Circuits whose (n_qubits, gate_off, n_gates) agree share one schedule. */
typedef struct {
  int32_t count;
  const int32_t* n_qubits;
  const int64_t* gate_off;
  const int32_t* n_gates;
  const int64_t* param_off;
  const int64_t* state_off;
} tq_batch;

/* State-vector execution options (NULL = defaults: fused, autotuned shapes).
 *   mode:      0 = fused (gates grouped into LDS-tile stages, one HBM sweep per stage),
 *              1 = plain (one HBM sweep per gate). Batches of circuits of uneven size and
 *              structure run best as a compiled batch (tq_svb_*, below).
 *   tile_bits: local qubits per fused tile (0 = default 12), 1..14.
 *   reg_bits:  amplitude-index bits held in registers per thread, 1..5 (0 = default 4).
 *   coal_bits: low index bits always kept local for coalesced HBM access (0 = default 4). */
typedef struct {
  int32_t mode;
  int32_t tile_bits;
  int32_t reg_bits;
  int32_t coal_bits;
} tq_sv_opts;

typedef struct tq_ctx tq_ctx;

/* Context on HIP device `device`. Owns schedule caches, the autotune table and scratch. */
tq_status tq_ctx_create(int device, tq_ctx** out);
void tq_ctx_destroy(tq_ctx* ctx);
/* Thread-local description of the last failure (empty string if none). */
const char* tq_last_error(void);
int tq_version(void);
/* HIP_VERSION the library was compiled with, and hipRuntimeGetVersion() of the runtime it
 * is bound to in this process (-1 if that call fails; no device needed). Kernels built by
 * a newer toolchain are not supported on an older runtime: callers must not use the
 * library when runtime < build. */
int tq_hip_build_version(void);
int tq_hip_runtime_version(void);

/* Sec. 3.1: apply every circuit of the batch to its state in place (|psi> <- U |psi>).
 * The caller fills d_states beforehand (|0..0> or its own vector: the library does not
 * normalise it). d_params holds real angles-parameters of the dtype's precision.
 * n_params[i] (may be NULL: then unchecked) bounds the parameter indices of circuit i.
 * Errors: TQ_EINVAL (bad op / qubit / duplicate qubit / parameter index >= n_params[i]),
 * TQ_ENOTSUP (n < 1 or n > 34). */
tq_status tq_sv_apply(tq_ctx* ctx, tq_dtype dt, const tq_batch* batch, const tq_gate* gates,
                      const int32_t* n_params, const void* d_params, void* d_states,
                      const tq_sv_opts* opts, void* stream);

/* Sec. 3.1 from the default start: every circuit's state becomes U |basis> (basis = 0 is the
 * paper's |0..0>); d_states is written, never read. The same result as tq_sv_init followed
 * by tq_sv_apply with the same arguments, with one HBM pass fewer: in fused mode the first
 * stage forms |basis> itself (plain mode and gate lists without a stage prepare the state
 * first). Errors: those of tq_sv_apply, and TQ_EINVAL if basis is outside [0, 2^n) for any
 * circuit. */
tq_status tq_sv_run(tq_ctx* ctx, tq_dtype dt, const tq_batch* batch, const tq_gate* gates,
                    const int32_t* n_params, const void* d_params, int64_t basis, void* d_states,
                    const tq_sv_opts* opts, void* stream);

/* Writes the computational basis state |basis> into every circuit's state (the default
 * initial state of Sec. 3.1 is basis = 0). Errors: TQ_EINVAL if basis is outside [0, 2^n). */
tq_status tq_sv_init(tq_ctx* ctx, tq_dtype dt, const tq_batch* batch, int64_t basis, void* d_states,
                     void* stream);

/* Shape of the schedule tq_sv_apply uses for one circuit structure (opts->mode 0 or 1), or
 * of the reverse-sweep schedule tq_sv_backward uses (opts->mode 2). Host only: with a
 * context a forward schedule is built and cached (with its device tables) as tq_sv_apply
 * does; with ctx == NULL, or in mode 2, it is built on the host, measured and dropped.
 * out[0] = HBM sweeps (kernel launches: stages in fused and reverse modes, ops in plain
 * mode), out[1] = scheduled ops after fusion, out[2] = register phases,
 * out[3] = LDS exchanges, out[4] = tile bits used, out[5] = register bits used,
 * out[6] = real flops per amplitude summed over ops (14 per 2x2, 6 per diagonal, 0 for
 * CNOT/CZ), out[7] = one-qubit matrices built per circuit. */
tq_status tq_sv_plan_info(tq_ctx* ctx, tq_dtype dt, int32_t n_qubits, const tq_gate* gates,
                          int32_t n_gates, const tq_sv_opts* opts, int64_t out[8]);

/* Sec. 4 cost: d_out[i * n_obs + o] = sum over terms with obs == o of
 * coeff * <psi_i| Z-string |psi_i> (real, written in the dtype's real precision). Each
 * thread sums |psi|^2 with the terms' signs over its own amplitudes (16 per 2^12-amplitude
 * chunk) in the state's precision; all further accumulation (over threads, work-groups and
 * terms) is in double with a fixed order, so repeated calls are bitwise equal. Terms name
 * qubits (bit q = qubit q). */
tq_status tq_expval(tq_ctx* ctx, tq_dtype dt, const tq_batch* batch, const void* d_states,
                    const tq_zterm* terms, int32_t n_terms, int32_t n_obs, void* d_out,
                    void* stream);

/* One Pauli string of an observable: coeff * prod_q P_q added to output `obs`, with P_q = X
 * where only bit q of x_mask is set, Z where only bit q of z_mask is set, Y where both are,
 * I elsewhere (bit q = qubit q). 32 bytes. */
typedef struct {
  uint64_t x_mask;
  uint64_t z_mask;
  double coeff;
  int32_t obs;
  int32_t _pad;
} tq_pauli_term;

/* Sec. 4 cost and Sec. 5.1.1 expectation values for Pauli strings with X, Y and Z factors:
 * d_out[i * n_obs + o] = sum over terms with obs == o of coeff * <psi_i| P |psi_i> (real for
 * the Hermitian P; written in the dtype's real precision). Each amplitude is read once per
 * distinct x_mask among the terms; sums are fixed-order double trees (bitwise repeatable).
 * A general Hermitian observable on a few qubits is a real combination of such strings
 * (its Pauli decomposition). Errors as tq_expval. */
tq_status tq_expval_pauli(tq_ctx* ctx, tq_dtype dt, const tq_batch* batch, const void* d_states,
                          const tq_pauli_term* terms, int32_t n_terms, int32_t n_obs, void* d_out, void* stream);

/* Host only: Pauli decomposition of a Hermitian matrix `herm` (2^k x 2^k complex, row-major,
 * interleaved doubles; row index with qubits[0] as its most significant bit) on the k <= 6
 * listed qubits: H = sum_P c_P P, c_P = Tr(P H) / 2^k. Writes the strings with |c_P| > tol as
 * terms of output `obs` to `out` (capacity `cap`; NULL to count) and returns their number,
 * or -1 (tq_last_error) on bad arguments or too small a capacity. With tq_expval_pauli this
 * gives <psi|H|psi> for a general Hermitian observable. */
int32_t tq_pauli_decompose(const double* herm, int32_t k, const int32_t* qubits, double tol, int32_t obs,
                           tq_pauli_term* out, int32_t cap);

/* Sec. 5.1.1 probability measurement: d_out[i * 2^n_sel + y] = probability that the listed
 * qubits read y (qubits[0] is the most significant bit of y), i.e. the sum of |psi_i|^2 over
 * every other qubit (the state is used as given, not normalised). 1 <= n_sel <= 24, at most
 * 32 other qubits; dtype's real precision, summed in double in a fixed order. Errors:
 * TQ_EINVAL (qubit outside the register or listed twice), TQ_ENOTSUP. */
tq_status tq_probs(tq_ctx* ctx, tq_dtype dt, const tq_batch* batch, const void* d_states, const int32_t* qubits,
                   int32_t n_sel, void* d_out, void* stream);

/* tq_expval for callers that cannot allocate (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): no context, no allocation, no synchronisation.
 * `count` circuits of n_qubits qubits whose states start at d_states + i * state_stride
 * (amplitudes; state_stride >= 2^n_qubits); at most 64 terms; d_out as tq_expval. The term
 * table and reduction partials live in a static 8 MiB device array per GPU (held until the
 * process ends); requests needing more (very many circuits) fail with TQ_EWORKSPACE. Every
 * call on a GPU shares that array, so calls that overlap on one GPU (other streams or host
 * threads at the same time) race; calls ordered on one stream do not. */
tq_status tq_expval_noalloc(tq_dtype dt, int32_t n_qubits, int32_t count, int64_t state_stride,
                            const void* d_states, const tq_zterm* terms, int32_t n_terms, int32_t n_obs,
                            void* d_out, void* stream);

/* Gradient of L = sum_i sum_o d_grad_out[i*n_obs+o] * <O_o>_i with respect to every
 * circuit's parameters, by one reverse (adjoint) sweep per circuit (Sec. 4: the values equal
 * the parameter-shift gradients of Sec. 4.2; the paper's backpropagation of Sec. 4.1 keeps
 * every intermediate state, the sweep keeps two). d_states holds the final states as left by
 * tq_sv_apply (read only). In the caller's workspace psi is copied, lambda = sum_o w_o O_o
 * psi, then for each gate in reverse psi <- U^dag psi, g += 2 Re<lambda| dU psi>,
 * lambda <- U^dag lambda. d_grad[param_off[i] + k] receives dL/d params_i[k] (overwritten,
 * dtype's real precision); gradients of all occurrences of a parameter are summed with
 * their pscale factors. d_grad_out is [count][n_obs] in the dtype's real precision.
 * d_work (device, work_bytes bytes, owned by the caller, contents need not be initialised)
 * must hold at least tq_sv_backward_workspace(...) bytes for the same arguments: psi and
 * lambda copies of the largest run of circuits sharing a gate list, their gate matrices and
 * gradient partial sums. Errors as tq_sv_apply / tq_expval, and TQ_EWORKSPACE (d_work NULL
 * or too small). The call neither allocates nor synchronises once the size query has been
 * made for the same gate lists, terms and batch offsets (the query builds and caches the
 * schedules and device tables the call uses). */
int64_t tq_sv_backward_workspace(tq_ctx* ctx, tq_dtype dt, const tq_batch* batch, const tq_gate* gates,
                                 const int32_t* n_params, const tq_zterm* terms, int32_t n_terms, int32_t n_obs,
                                 const tq_sv_opts* opts); /* bytes, or -1 on error (tq_last_error) */
tq_status tq_sv_backward(tq_ctx* ctx, tq_dtype dt, const tq_batch* batch, const tq_gate* gates,
                         const int32_t* n_params, const void* d_params, const void* d_states,
                         const tq_zterm* terms, int32_t n_terms, int32_t n_obs,
                         const void* d_grad_out, void* d_grad, const tq_sv_opts* opts,
                         void* d_work, int64_t work_bytes, void* stream);

/* One parameter update of a training loop (Sec. 4: the cost f is minimised by gradient
 * steps on the circuit parameters), on the device: kind 0 = gradient descent
 * p -= lr * g; kind 1 = Adam (Kingma and Ba) with bias correction for the 1-based step t,
 * moments d_m, d_v (zero before step 1) updated in place. Arrays of n reals of the dtype's
 * precision; arithmetic in double. Errors: TQ_EINVAL. */
tq_status tq_optimizer_step(tq_dtype dt, int32_t kind, void* d_params, const void* d_grad, void* d_m, void* d_v,
                            int32_t t, double lr, double beta1, double beta2, double eps, int64_t n, void* stream);

/* tq_sv_backward for observables that are real combinations of Pauli strings with X, Y and
 * Z factors (at most 16 terms): lambda = sum_o w_o O_o psi is formed from the strings
 * directly, the reverse sweep is the same. The workspace is the size tq_sv_backward_workspace
 * reports for the same batch and gate lists (the terms do not change it). Errors as
 * tq_sv_backward. */
tq_status tq_sv_backward_pauli(tq_ctx* ctx, tq_dtype dt, const tq_batch* batch, const tq_gate* gates,
                               const int32_t* n_params, const void* d_params, const void* d_states,
                               const tq_pauli_term* terms, int32_t n_terms, int32_t n_obs, const void* d_grad_out,
                               void* d_grad, const tq_sv_opts* opts, void* d_work, int64_t work_bytes,
                               void* stream);

/* ---------------------------------------------------------------------------------------
 * Compiled batches. The paper compiles a circuit once and evaluates it many times with new
 * parameters (Sec. 2, reusable objects), and runs one circuit over a batch of inputs with
 * vmap (Sec. 5.3). A tq_svb is that compiled form for a whole batch of circuits, which may
 * differ in size and structure: every circuit's fused schedule, and work lists in which one
 * kernel per stage level runs the tiles of all circuits that have that level (largest work
 * items first), so small circuits share launches with large ones. Forward = |0..0> (or the
 * caller's state) + gate application + expectation values; backward = the adjoint sweep of
 * every circuit. With opts.graph = 1 each call's launch sequence is captured once per set of
 * buffer pointers (on the second call with those pointers) and replayed as a HIP graph.
 * Device buffers owned by the tq_svb (gate matrices, adjoint working states, partial sums)
 * are allocated on first use and released by tq_svb_destroy.
 * ------------------------------------------------------------------------------------- */
typedef struct tq_svb tq_svb;

/* Zero fields take defaults. tile/reg/coal bits as in tq_sv_opts, for the forward stages
 * and (adj_*) for the reverse sweep (defaults 12/4 for TQ_C64, 11/3 for TQ_C128).
 * init: 0 = forward starts every circuit from |0..0> (written by the library), 1 = from the
 * caller's states. graph: 1 = capture and replay HIP graphs. */
typedef struct {
  int32_t tile_bits, reg_bits, coal_bits;
  int32_t adj_tile_bits, adj_reg_bits, adj_coal_bits;
  int32_t init;
  int32_t graph;
} tq_svb_opts;

/* Host-side compile of a batch (gates, n_params and terms are copied; nothing is launched).
 * Terms and n_obs are shared by all circuits. Errors as tq_sv_apply / tq_expval. */
tq_status tq_svb_create(tq_ctx* ctx, tq_dtype dt, const tq_batch* batch, const tq_gate* gates,
                        const int32_t* n_params, const tq_zterm* terms, int32_t n_terms, int32_t n_obs,
                        const tq_svb_opts* opts, tq_svb** out);
void tq_svb_destroy(tq_svb* b);

/* d_states at the batch's state offsets are overwritten with the final states; d_out
 * ([count][n_obs], may be NULL to skip) receives the expectation values as tq_expval. */
tq_status tq_svb_forward(tq_ctx* ctx, tq_svb* b, const void* d_params, void* d_states, void* d_out,
                         void* stream);

/* Adjoint gradients as tq_sv_backward: d_states holds the final states (read only),
 * d_grad_out is [count][n_obs], d_grad at the parameter offsets is overwritten. */
tq_status tq_svb_backward(tq_ctx* ctx, tq_svb* b, const void* d_params, const void* d_states,
                          const void* d_grad_out, void* d_grad, void* stream);

/* Autotuner: times the forward (which = 0; overwrites d_states) or backward (which = 1;
 * d_states read only, unit upstream gradients) pass for every candidate shape (tile bits,
 * register bits) on the device, `reps` timed runs each after one warm-up, keeps the fastest
 * in the tq_svb and in the context (later tq_svb_create calls for the same batch structure
 * start from it), and reports it in *best (may be NULL) with its mean time in *best_ms.
 * Synchronises the stream. */
tq_status tq_svb_autotune(tq_ctx* ctx, tq_svb* b, const void* d_params, void* d_states, int32_t which,
                          int32_t reps, void* stream, tq_svb_opts* best, double* best_ms);

/* out[0] forward stage levels, [1] forward work items (tiles over all levels), [2] reverse
 * levels, [3] reverse work items (0 before the first backward call), [4] graphs captured,
 * [5] graph replays, [6] forward tile bits, [7] forward register bits. */
tq_status tq_svb_info(const tq_svb* b, int64_t out[8]);

/* Persistence of the autotune table (Sec. 2: compiled objects reused across runs), host only.
 * tq_ctx_export_tuning writes the context's tuned shapes, its own and imported ones, to `buf`
 * (capacity `cap` bytes; NULL to query the size) and returns the byte count, or -1
 * (tq_last_error) on a NULL context or too small a capacity. Layout: a 16-byte header
 * ("TQTU", version 1, record count, 0) then 40-byte records: a 32-byte digest of (batch
 * structure, pass), tile bits, register bits. tq_ctx_import_tuning reads such a buffer into
 * a context: later tq_svb_create calls whose structure digest matches start from the
 * imported shape (a shape changes speed only; one the structure cannot take falls back to
 * the defaults). TQ_EINVAL on a malformed buffer or a shape outside tile 1..14 / register
 * 1..5, in which case nothing is imported. */
int64_t tq_ctx_export_tuning(const tq_ctx* ctx, void* buf, int64_t cap);
tq_status tq_ctx_import_tuning(tq_ctx* ctx, const void* buf, int64_t len);

/* ---------------------------------------------------------------------------------------
 * Tensor-network mode (Sec. 3.2). A closed or open network of leaf tensors whose indices all
 * have dimension 2; an index may be shared by any number of tensors (hyperedge, Sec. 3.2.1).
 * A tensor of rank r is 2^r complex numbers, its first index the most significant bit.
 * The contraction order is a binary tree (Sec. 3.2.2) given in SSA form: step s contracts
 * ids pairs[2s], pairs[2s+1] (ids < n_leaves are leaves, n_leaves + s is the result of
 * step s). Sliced indices (Sec. 3.2.3) are fixed to each of their 2^n_sliced assignments;
 * the value is the sum of the sub-network values. Leaves are packed in one device buffer,
 * leaf i at complex offset tq_tn_leaf_offset(plan, i), in full (unsliced) size.
 * ------------------------------------------------------------------------------------- */
typedef struct tq_tn_plan tq_tn_plan;

typedef struct {
  int32_t n_leaves;
  const int32_t* leaf_rank;  /* [n_leaves] */
  const int32_t* leaf_inds;  /* concatenated index ids, leaf by leaf, first = most significant */
  const int32_t* pairs;      /* [2 * (n_leaves - 1)] SSA tree */
  int32_t n_sliced;
  const int32_t* sliced;     /* index ids fixed per slice (0..20) */
  int32_t n_out;             /* open indices of the result, in the order wanted (0: scalar) */
  const int32_t* out_inds;
  int32_t dtype;             /* tq_dtype */
  int64_t slice_group;       /* slices contracted together per launch sequence (0 = auto) */
  int64_t mem_budget;        /* bytes of workspace the auto slice group may use (0 = 4 GiB) */
  int32_t store_policy;      /* TQ_TN_RECOMPUTE, TQ_TN_STORE or TQ_TN_AUTO, below */
  int32_t _pad;
} tq_tn_desc;

/* What the reverse pass does for the forward's intermediate tensors. The paper's
 * backpropagation (Sec. 4.1) stores them; recomputing them trades one extra forward pass for
 * memory when the slices cannot all be held at once.
 *   TQ_TN_RECOMPUTE: tq_tn_backward recomputes the forward inside the call (any slice group).
 *   TQ_TN_STORE: tq_tn_backward reuses the intermediates that the immediately preceding
 *     tq_tn_contract of the same plan and leaves left in the same workspace (which must then
 *     have the backward size, tq_tn_workspace(plan, 1)); the plan must run all slices as one
 *     group within mem_budget, else tq_tn_plan_create fails with TQ_ENOTSUP.
 *   TQ_TN_AUTO: store when all slices fit mem_budget as one group, else recompute.
 * The batched calls (tq_tn_*_batch) always recompute. */
enum { TQ_TN_RECOMPUTE = 0, TQ_TN_STORE = 1, TQ_TN_AUTO = 2 };

/* Host-side planning: classifies every step (batch / contracted / kept / summed-out
 * indices), picks its kernel (direct bit-indexed contraction, or bit-permute + MFMA complex
 * GEMM, FP32 for complex64 and FP64 for complex128, when M, N, K are all large), sizes the
 * workspace, then copies the step tables to the context's device. With ctx == NULL the plan
 * is built on the host only: the query calls below (stores, segments, leaf offsets,
 * workspace, info) work on it, and every call that would run it fails with TQ_EINVAL.
 * Errors: TQ_EINVAL if the tree does not use every leaf exactly once, an id is out of
 * range, or the result's open indices differ from out_inds as a set. */
tq_status tq_tn_plan_create(tq_ctx* ctx, const tq_tn_desc* desc, tq_tn_plan** out);
void tq_tn_plan_destroy(tq_tn_plan* plan);
/* 1 if tq_tn_backward of this plan reuses the forward's stored intermediates (the store
 * policy is in effect), 0 if it recomputes them, -1 for a NULL plan. */
int32_t tq_tn_plan_stores(const tq_tn_plan* plan);
/* Launch structure of a plan: out[0] forward segments (one launch sequence each: a fused run
 * of small steps, or one large step), out[1] of them fused runs, out[2] reverse segments,
 * out[3] of them fused runs (per slice group). */
tq_status tq_tn_plan_segments(const tq_tn_plan* plan, int64_t out[4]);
/* Complex elements of the packed leaf buffer, and leaf i's offset in it. */
int64_t tq_tn_leaf_elems(const tq_tn_plan* plan);
int64_t tq_tn_leaf_offset(const tq_tn_plan* plan, int32_t leaf);
/* Workspace bytes for tq_tn_contract (backward = 0) or tq_tn_backward (backward = 1). */
int64_t tq_tn_workspace(const tq_tn_plan* plan, int32_t backward);
/* Plan statistics: out[0] steps, [1] direct steps, [2] GEMM steps, [3] slices,
 * [4] slice group, [5] real flops per contraction (8 per complex multiply-add, all slices),
 * [6] real flops in GEMM steps, [7] largest intermediate (complex elements, per slice). */
tq_status tq_tn_plan_info(const tq_tn_plan* plan, int64_t out[8]);

/* Step (e) of Sec. 3.2: d_out (2^n_out complex) = the network's value, summed over slices.
 * d_leaves is the packed leaf buffer (read only). */
tq_status tq_tn_contract(tq_ctx* ctx, const tq_tn_plan* plan, const void* d_leaves, void* d_out, void* d_work,
                         int64_t work_bytes, void* stream);

/* Reverse pass over the tree (Sec. 4.1, backpropagation through the contraction):
 * d_grad_leaves (packed like the leaves) receives, for every leaf, its environment scaled
 * by the upstream value: sum over the output entries o of d_grad_out[o] * dT[o]/dL
 * (holomorphic derivative of the multilinear value T). For a real loss
 * l = Re sum_o conj(g_o) T_o pass d_grad_out = g; dl/dtheta is then
 * Re sum_leaf sum_x d_grad_leaves[x] * dL[x]/dtheta. The forward's intermediates are
 * recomputed inside the call, or reused from the workspace under the store policy
 * (tq_tn_desc.store_policy). Errors: TQ_EWORKSPACE if work_bytes < tq_tn_workspace(plan, 1). */
tq_status tq_tn_backward(tq_ctx* ctx, const tq_tn_plan* plan, const void* d_leaves, const void* d_grad_out,
                         void* d_grad_leaves, void* d_work, int64_t work_bytes, void* stream);

/* Many networks at once (e.g. one light-cone network per measured edge). Arrays of length n
 * hold each network's plan, packed leaves, output (value: 2^n_out complex; backward: the
 * packed leaf environments), workspace and its size (tq_tn_workspace(plan, 0 or 1)). Plans
 * without slices whose passes are short runs of small steps execute together in one launch,
 * one work-group per network; the others run as tq_tn_contract / tq_tn_backward would.
 * Plans in one launch must share a dtype. The upload of the network table is stream-ordered. */
tq_status tq_tn_contract_batch(tq_ctx* ctx, int32_t n, const tq_tn_plan* const* plans,
                               const void* const* d_leaves, void* const* d_out, void* const* d_work,
                               const int64_t* work_bytes, void* stream);
tq_status tq_tn_backward_batch(tq_ctx* ctx, int32_t n, const tq_tn_plan* const* plans,
                               const void* const* d_leaves, const void* const* d_grad_out,
                               void* const* d_grad_leaves, void* const* d_work,
                               const int64_t* work_bytes, void* stream);

/* Leaves of a circuit network from the circuit parameters (Sec. 3.2.1: state, gate and
 * observable tensors, with conjugate copies for the bra half). kind per leaf: 0 constant
 * (const_vals[const_off ..], complex128 interleaved), 1 one-qubit gate [out, in],
 * 2 one-qubit diagonal gate over its wire index, 3 two-qubit diagonal gate over its two wire
 * indices, 4 two-qubit gate [out_a, out_b, in_a, in_b]; conj = 1 for the bra copy.
 * flip (anti-diagonal reduction, Sec. 3.2.1): the leaf stores entry e ^ flip of its kind's
 * tensor at element e (bit 0 = its last listed index), so an anti-diagonal gate (X, or Y as
 * a diagonal then X) needs no tensor: the wire's later tensors read that index flipped.
 * Must be below 2^rank. */
typedef struct {
  int32_t kind;
  int32_t gate;
  int16_t conj;
  uint16_t flip;
  int32_t const_off;
} tq_tn_leaf;

tq_status tq_tn_build_leaves(tq_ctx* ctx, const tq_tn_plan* plan, const tq_gate* gates, int32_t n_gates,
                             const tq_tn_leaf* leaves, const double* const_vals, int32_t n_const,
                             const void* d_params, void* d_leaves, void* stream);

/* Chain rule from leaf environments to circuit parameters:
 * d_grad_params[p] = Re sum over leaves built from a gate using p, of
 * sum_x d_grad_leaves[x] * d(leaf)[x]/d(params[p]) (overwrites n_params entries). */
tq_status tq_tn_param_grad(tq_ctx* ctx, const tq_tn_plan* plan, const tq_gate* gates, int32_t n_gates,
                           const tq_tn_leaf* leaves, const void* d_params, int32_t n_params,
                           const void* d_grad_leaves, void* d_grad_params, void* stream);

/* The two calls above for n networks at once, each in one launch (the same results, bit for
 * bit, as n single calls). Arrays of length n hold each network's arguments as the single
 * call takes them (host arrays: gates, leaves, const_vals; device buffers: params, leaves,
 * grad_leaves, grad_params). Every plan of one call must have the same dtype. All networks
 * are checked before anything is launched; an error names the first network whose arguments
 * fail the single call's checks. The networks then launch in chunks of 256, each chunk's
 * table uploaded in stream order, like tq_tn_contract_batch's. */
tq_status tq_tn_build_leaves_batch(tq_ctx* ctx, int32_t n, const tq_tn_plan* const* plans,
                                   const tq_gate* const* gates, const int32_t* n_gates,
                                   const tq_tn_leaf* const* leaves, const double* const* const_vals,
                                   const int32_t* n_const, const void* const* d_params, void* const* d_leaves,
                                   void* stream);
tq_status tq_tn_param_grad_batch(tq_ctx* ctx, int32_t n, const tq_tn_plan* const* plans,
                                 const tq_gate* const* gates, const int32_t* n_gates, const tq_tn_leaf* const* leaves,
                                 const void* const* d_params, const int32_t* n_params,
                                 const void* const* d_grad_leaves, void* const* d_grad_params, void* stream);

/* ---------------------------------------------------------------------------------------
 * Cost-model MLP (ranks contraction trees by predicted runtime; Sec. 3.2.2 ranks them by
 * FLOPs, and Sec. 6.6 notes that small pairwise steps make runtime and FLOPs disagree).
 * x -> tanh(W_1 x + b_1) -> ... -> tanh(W_{L-1} h + b_{L-1}) -> W_L h + b_L, float32, one
 * scalar output (sizes[n_layers] must be 1). Parameters are packed layer by layer as
 * W_l [sizes[l+1]][sizes[l]] row-major followed by b_l [sizes[l+1]]. Inputs are [batch][sizes[0]]
 * row-major. Reductions over the batch run in a fixed order (repeatable bitwise).
 * ------------------------------------------------------------------------------------- */
typedef struct {
  int32_t n_layers;  /* 1..8 */
  int32_t sizes[9];  /* sizes[0] = input features, ..., sizes[n_layers] = 1; each 1..4096 */
} tq_mlp_desc;

/* Number of packed parameters, and workspace bytes for a batch (-1 on a bad descriptor). */
int64_t tq_mlp_param_count(const tq_mlp_desc* desc);
int64_t tq_mlp_workspace(const tq_mlp_desc* desc, int32_t batch);

/* d_y[b] = MLP(d_x[b]). Errors: TQ_EINVAL, TQ_EWORKSPACE. */
tq_status tq_mlp_forward(tq_ctx* ctx, const tq_mlp_desc* desc, const float* d_params, const float* d_x,
                         int32_t batch, float* d_y, void* d_work, int64_t work_bytes, void* stream);

/* One Adam step (Kingma and Ba, bias-corrected; t is the 1-based step count) on the mean
 * squared error L = mean_b (MLP(x_b) - y_b)^2: d_params, d_m, d_v (first and second moments,
 * zero before step 1) are updated in place. d_loss (may be NULL) receives L before the
 * update, d_grad (may be NULL) dL/dparams. */
tq_status tq_mlp_train_step(tq_ctx* ctx, const tq_mlp_desc* desc, float* d_params, float* d_m, float* d_v,
                            int32_t t, float lr, float beta1, float beta2, float eps, const float* d_x,
                            const float* d_y, int32_t batch, float* d_loss, float* d_grad, void* d_work,
                            int64_t work_bytes, void* stream);

/* ---------------------------------------------------------------------------------------
 * Attainable peaks. The rooflines the kernels are graded against (HBM bandwidth for the
 * sweeps, vector and matrix-core rates for the stage and contraction kernels) are quoted
 * both against the datasheet and against what fixed kernels reach on the device at hand.
 * ------------------------------------------------------------------------------------- */

/* Enqueues one probe launch on `stream` and sets *work to the work it does; the caller times
 * the launch with events on that stream. kind 0: stream copy, the first half of the device
 * buffer d_buf is copied to the second half (one 16-byte vector per thread), *work = bytes
 * (half read plus half written). kind 4: stream read of all of d_buf, *work = bytes; it
 * writes nothing unless the buffer's values sum to -1 in a thread's share, and then only the
 * first float of d_buf. For kinds 0 and 4, bytes is a positive multiple of 32 KiB, at most
 * 8 TiB. kind 1: FP32 fused multiply-add chains, non-packed (2048 x 256 threads x iters x 8
 * FMAs; *work in flops). kind 2: FP32 16x16x4 matrix-core accumulations (8192 waves x iters
 * x 8, 2048 flops each). kind 3: the same with FP64. Kinds 1-3 write one value per thread to
 * d_buf, which must hold 2048 x 256 floats (kinds 1, 2) or doubles (kind 3). Errors:
 * TQ_EINVAL (null pointer, unknown kind, iters < 1), TQ_ESIZE (buffer too small, or not a
 * multiple of 32 KiB for kinds 0 and 4). */
tq_status tq_peak_probe(int32_t kind, void* d_buf, uint64_t bytes, int32_t iters, double* work, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* LIBTQ_TQ_H_ */
