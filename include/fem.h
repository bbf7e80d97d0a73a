/*
 * fem.h -- C ABI of the MI355X (gfx950) Free-Energy Machine hot path.
 *
 * The Free-Energy Machine (FEM; Shen et al., arXiv 2412.09285) minimises,
 * for R independent replicas at once, the variational mean-field free energy
 *     F = U_MF - S_MF / beta
 * (supplementary "Derivation of variational mean-field free energy
 * formulations") by gradient steps with Adam on the fields h while beta is
 * annealed upwards (Methods, "Different annealing schedules"), then rounds
 * every replica to a configuration and keeps the best one (Results,
 * "Free-Energy Machine", the two read-out equations).
 *
 * Conventions (fixed for every call):
 *  - Ids are 0-based.  Graphs are given as undirected edge lists, each edge
 *    {u,v} once; energies sum over ordered pairs (each edge both ways), which
 *    is the convention under which the paper's explicit gradients are the
 *    derivatives of F.  Reported integer cuts count each edge once.
 *  - MaxCut and Max-k-SAT carry one logit per variable (P = sigmoid(h), the
 *    paper's q = 2 reduction); balanced min-cut carries q logits per node
 *    (softmax).  Q below is 1 or q accordingly.
 *  - Field-shaped device/host buffers are float32, node-row and replica
 *    contiguous: h[n][R] (Q = 1) or h[n][R][q], state index fastest.
 *  - Configurations sigma are int32 [R][n] (replica-major) with states
 *    0..q-1; for one-logit problems sigma_i = 1 iff h_i > 0 (ties to 0).
 *  - For a batch of B instances (fem_batch_create) per-instance outputs are
 *    laid out [B][R] and node ids run over the concatenation of the parts.
 *
 * Ownership: host arrays passed in are borrowed for the duration of the call
 * (copied).  Problems and solvers own their device memory.  A pointer flagged
 * on_device is caller-owned device memory on the solver's device, accessed
 * only inside the call, ordered on the solver's stream.
 *
 * Errors: every call returns a fem_status; nothing throws, aborts or exits.
 * The text of the last failure on the calling thread is fem_last_error().
 * Kernels run asynchronously: fem_step / fem_run only enqueue work, and a
 * failure inside a kernel surfaces at the next call that synchronises
 * (fem_sync and every getter).  A solver is not thread-safe; distinct
 * solvers may run concurrently on distinct streams.
 */
#ifndef FEM_H
#define FEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FEM_OK = 0,
    FEM_E_INVAL = -1,        /* malformed argument or input (message says which) */
    FEM_E_NOMEM = -2,        /* host or device allocation failed */
    FEM_E_HIP = -3,          /* HIP runtime error (message holds hipGetErrorString) */
    FEM_E_STATE = -4,        /* call not valid in the object's current state */
    FEM_E_NUMERIC = -5,      /* a non-finite energy or field was detected */
    FEM_E_UNSUPPORTED = -6   /* valid request outside what this build supports */
} fem_status;

enum { FEM_MAXCUT = 0, FEM_BMINCUT = 1, FEM_MAXSAT = 2 };
/* beta schedules: linear in beta; exponential (Methods); inverse-proportional,
 * i.e. linear in temperature (Methods).  All give beta(0) = beta_min and
 * beta(steps-1) = beta_max. */
enum { FEM_SCHED_LINEAR = 0, FEM_SCHED_EXP = 1, FEM_SCHED_INVPROP = 2 };
/* storage type of the marginal copy that neighbours gather */
enum { FEM_F32 = 0, FEM_BF16 = 1 };

const char* fem_status_str(int status);
const char* fem_last_error(void);
/* ABI version, bumped on any incompatible change of this header. */
int32_t fem_abi_version(void);

typedef struct fem_problem fem_problem;   /* immutable, device resident */
typedef struct fem_solver fem_solver;     /* R replicas: h, Adam moments, marginals, t */

/* ---------------------------------------------------------------- problems */

/* MaxCut (Results, "Applications to the Maximum-Cut problem"):
 * E(sigma) = -sum_{(i,j) in E} W_ij [1 - delta(sigma_i, sigma_j)].
 * u, v: n_edges endpoints (host, 0 <= u,v < n, u != v, no duplicate pair);
 * w: host weights or NULL for all +1.  Self-loops, duplicate edges,
 * out-of-range ids, non-finite weights and n < 1 give FEM_E_INVAL.
 * Device memory: the symmetric CSR (8-byte row offsets, 8-byte entries) and,
 * when every weight is +1 or -1, a second 4-byte copy of the entries (column
 * and sign) that the step kernel reads. */
fem_status fem_maxcut_create(int device, int32_t n, int64_t n_edges, const int32_t* u,
                             const int32_t* v, const float* w, fem_problem** out);

/* MaxCut on a dense weight matrix: complete or near-complete graphs such as
 * the all-to-all K2000 benchmark (Results, "Applications to the Maximum-Cut
 * problem").  W: host, n x n row-major float, symmetric with zero diagonal
 * and finite entries (FEM_E_INVAL otherwise); n <= 32768 (FEM_E_UNSUPPORTED).
 * With explicit gradients the step forms the field product W m on the
 * matrix cores (float32 marginals; a bfloat16 marginal copy gives
 * FEM_E_UNSUPPORTED at solver creation); read-out, evaluation and the
 * manipulated gradients use the sparse structure of W's nonzeros, which the
 * problem also holds.  Device memory: W zero-padded to a multiple of 128 rows
 * and columns (float) plus that structure.  Dense problems are not batched
 * (fem_batch_create gives FEM_E_UNSUPPORTED). */
fem_status fem_maxcut_create_dense(int device, int32_t n, const float* W, fem_problem** out);

/* q-way balanced min-cut (Results, the bMinCut energy with the soft balance
 * term lambda * sum_i sum_{j != i} delta(sigma_i, sigma_j)).  Same edge rules
 * as MaxCut; weights must be > 0.  q must be one of 2, 4, 8, 16, 32 (other
 * q >= 2 give FEM_E_UNSUPPORTED).  lambda is a solver parameter. */
fem_status fem_bmincut_create(int device, int32_t n, int64_t n_edges, const int32_t* u,
                              const int32_t* v, const float* w, int32_t q, fem_problem** out);

/* bMinCut with node weights V_i (the community sizes of a coarsened graph,
 * Methods, multilevel bMinCut): the balance term becomes
 * lambda * sum_s [W_s^2 - sum_i V_i^2 delta(sigma_i, s)] with W_s the summed
 * weight of group s, and its mean-field form
 * lambda * sum_s [(sum_i V_i P_i(s))^2 - sum_i V_i^2 P_i(s)^2].  node_weight:
 * host, n entries, each >= 1 (FEM_E_INVAL otherwise, also for NULL); their
 * sum must not exceed 2^22 (FEM_E_UNSUPPORTED).  All weights 1 is the same
 * problem as fem_bmincut_create.  Group sizes reported by fem_eval_int are
 * then group weights W_s. */
fem_status fem_bmincut_create_weighted(int device, int32_t n, int64_t n_edges, const int32_t* u,
                                       const int32_t* v, const float* w, int32_t q,
                                       const int32_t* node_weight, fem_problem** out);

/* Max-k-SAT (Results, "Application to the Max k-SAT problem"): energy = number
 * of unsatisfied clauses.  DIMACS-style literals +(x+1) / -(x+1) on host;
 * clause_off has n_clauses+1 nondecreasing entries starting at 0.  A repeated
 * literal counts once; a clause holding x and not-x is always satisfied and is
 * dropped; an empty clause, a zero literal or an out-of-range variable gives
 * FEM_E_INVAL; a clause of more than 4 distinct variables gives
 * FEM_E_UNSUPPORTED. */
fem_status fem_maxsat_create(int device, int32_t n_vars, int64_t n_clauses,
                             const int64_t* clause_off, const int32_t* lits, fem_problem** out);

/* Block-diagonal union of n problems of one kind (and one q) on one device:
 * one solver then runs every instance in the same launches, with per-instance
 * energies, read-out and best replica.  The parts stay owned by the caller and
 * may be destroyed afterwards. */
fem_status fem_batch_create(int32_t n, fem_problem* const* parts, fem_problem** out);

/* kind, total nodes/variables, q (2 for one-logit kinds), directed adjacency
 * entries (2 x edges) or literal incidences, number of instances.  Any output
 * pointer may be NULL. */
fem_status fem_problem_info(const fem_problem* p, int32_t* kind, int32_t* n, int32_t* q,
                            int64_t* nnz, int32_t* n_instances);
/* node offsets of the instances, n_instances+1 entries (host). */
fem_status fem_problem_instance_offsets(const fem_problem* p, int32_t* offsets);
void fem_problem_destroy(fem_problem* p);

/* Locality order of a graph's nodes for the neighbour gathers (host only; an
 * implementation aid, not part of the method): reverse Cuthill-McKee (Cuthill
 * and McKee 1969, reversed as in George 1971), component by component, each
 * started from a pseudo-peripheral node found by repeated breadth-first
 * search (George and Liu 1979), neighbours visited by increasing degree, then
 * index.  order[k] (n entries, caller-owned) is the node placed at position
 * k; relabelling node order[k] as k before fem_*_create keeps most
 * neighbours within a band of rows, so on geometric or mesh-like graphs the
 * gathered rows stay in L2.  Results then come back in the new labels.
 * Edges as for fem_maxcut_create (no self-loops); FEM_E_INVAL otherwise. */
fem_status fem_graph_order(int32_t n, int64_t n_edges, const int32_t* u, const int32_t* v, int32_t* order);

/* ------------------------------------------------------------------ solver */
typedef struct {
    int32_t replicas;          /* R >= 1 */
    int32_t steps;             /* annealing length T >= 1 */
    int32_t schedule;          /* FEM_SCHED_* */
    double beta_min, beta_max; /* 0 < beta_min <= beta_max */
    double lr, adam_b1, adam_b2, adam_eps, weight_decay;   /* torch.optim.Adam semantics */
    double lambda;             /* bMinCut balance weight (lambda_max when ramped) */
    int32_t lambda_ramp;       /* 0: constant; 1: lambda(t) = lambda * t / (T-1) */
    int32_t marginal_dtype;    /* FEM_F32 | FEM_BF16 */
    int32_t energy_every;      /* per-replica U, S, F every k-th step (0 = never) */
    int32_t record_energies;   /* keep the energies of every evaluated step */
    int32_t eval_every;        /* anytime read-out every k steps (0 = only on request) */
    int32_t keep_grad;         /* keep the last gradient for fem_last_grad */
    int32_t optimizer;         /* FEM_OPT_ADAM | FEM_OPT_RMSPROP | FEM_OPT_SGD */
    double momentum;           /* RMSprop / SGD momentum */
    double rms_alpha;          /* RMSprop smoothing constant */
    double dampening;          /* SGD dampening */
    int32_t gradient;          /* FEM_GRAD_EXPLICIT | FEM_GRAD_MANIPULATED */
    double gamma_grad;         /* gamma_grad of the manipulated gradients */
    int32_t state_layout;      /* FEM_STATE_SEPARATE | FEM_STATE_INTERLEAVED */
} fem_params;

/* Device layout of the optimiser state (h and the two moments); it changes
 * no result, only how the step kernels stream it, and every getter and setter
 * keeps the [n][R] / [n][R][q] layout of each array.
 *  FEM_STATE_SEPARATE: three arrays.
 *  FEM_STATE_INTERLEAVED (default): the three rows of a node next to each
 *    other, one contiguous stream per node instead of three. */
enum { FEM_STATE_SEPARATE = 0, FEM_STATE_INTERLEAVED = 1 };

/* Gradient with respect to the fields (supplementary "The explicit gradient
 * formulations" and "The explicit gradients and manipulated gradients for the
 * benchmarking problems"):
 *  FEM_GRAD_EXPLICIT: the exact gradient of the mean-field free energy.
 *  FEM_GRAD_MANIPULATED: the paper's modified gradient, gamma_grad times the
 *    softmax chain rule applied to
 *      MaxCut:  c_i sum_j W_ij e_j(s) + (ln P_i(s) + 1)/beta, c_i = 1/sum_j|W_ij|;
 *      bMinCut: -c^f_i sum_j W_ij e_j(s) + lambda c^a_i [sum_j e_j(s) - e_i(s)]
 *               + (ln P_i(s) + 1)/beta, c^f_i = q/sum_j W_ij,
 *               c^a_i = q/sqrt(sum_j W_ij);
 *      Max-k-SAT: the explicit gradient (left unmodified by the paper);
 *    e_j is the one-hot read-out of node j (fem_round's rule) and a node
 *    without incident weight gets c = 0.  The marginal copy becomes that
 *    read-out (1 bit per replica for MaxCut, 1 byte for bMinCut), so
 *    marginal_dtype is ignored for those kinds.  Not the gradient of F: the
 *    per-replica energies are not formed, and energy_every must be 0
 *    (else FEM_E_UNSUPPORTED). */
enum { FEM_GRAD_EXPLICIT = 0, FEM_GRAD_MANIPULATED = 1 };

/* Optimisers, torch.optim semantics (the paper uses PyTorch's Adam, RMSprop
 * and SGD; Methods, "Hyperparameter tuning").  The Adam moments m1, m2 hold
 * RMSprop's momentum buffer and square average, or SGD's momentum buffer. */
enum { FEM_OPT_ADAM = 0, FEM_OPT_RMSPROP = 1, FEM_OPT_SGD = 2 };

/* Adam 0.9 / 0.999 / 1e-8, lr 0.1, no weight decay, linear beta 0.01 -> 5,
 * R = 16, T = 500, F32 marginals, energies every step, no recording;
 * RMSprop alpha 0.99, no momentum or dampening; explicit gradients,
 * gamma_grad 1; interleaved state layout. */
void fem_params_default(fem_params* p);

/* hip_stream: a hipStream_t on the problem's device (NULL = the null stream).
 * The solver keeps a reference to the problem: fem_problem_destroy may be
 * called while solvers still use it (the memory is released with the last). */
fem_status fem_solver_create(const fem_problem* p, const fem_params* prm, void* hip_stream,
                             fem_solver** out);
void fem_solver_destroy(fem_solver* s);

/* Initial fields h0 ([n][R] or [n][R][q] float32, host or device).  Resets the
 * Adam moments to zero, the step counter t to 0, the anytime bests, and
 * recomputes the marginal copy. */
fem_status fem_set_fields(fem_solver* s, const float* h, int on_device);

/* Full optimiser state: fields h, Adam moments m1, m2 (all in the layout of
 * h, float32, host or device) and the step counter t (0 <= t <= T); the
 * marginal copy is recomputed.  Resumes an anneal from any state. */
fem_status fem_set_adam_state(fem_solver* s, const float* h, const float* m1, const float* m2,
                              int32_t t, int on_device);

/* Enqueue n_steps annealing steps t -> t+1 (t + n_steps <= T).  Step t uses
 * beta(t), lambda(t) and Adam step count t+1; its gradient and energies are
 * evaluated at h(t). */
fem_status fem_step(fem_solver* s, int32_t n_steps);
/* Enqueue the remaining steps up to T as one captured HIP graph (replayed on
 * later calls from the same t). */
fem_status fem_run(fem_solver* s);
/* Enqueue steps [t, t_end) as one captured HIP graph. */
fem_status fem_run_until(fem_solver* s, int32_t t_end);
/* Capture (and instantiate) the graph of steps [t, t_end) without running it,
 * so that a later fem_run_until(s, t_end) from the same t only launches it.
 * Needs a non-null stream. */
fem_status fem_capture(fem_solver* s, int32_t t_end);
fem_status fem_sync(fem_solver* s);
/* current step counter t */
fem_status fem_get_step(const fem_solver* s, int32_t* t);

fem_status fem_get_fields(fem_solver* s, float* h, int on_device);
/* gradient dF/dh of the last step (needs keep_grad), layout of h. */
fem_status fem_last_grad(fem_solver* s, float* g, int on_device);
/* U, S, F of the last evaluated step, [B][R] each (any may be NULL).  Gives
 * FEM_E_STATE if no step evaluated energies, FEM_E_NUMERIC if a value is not
 * finite. */
fem_status fem_energies(fem_solver* s, double* U, double* S, double* F);
/* energies recorded at steps t0, t0+k, ... (record_energies), count entries of
 * [B][R] each. */
fem_status fem_energy_history(fem_solver* s, int32_t first, int32_t count, double* U,
                              double* S, double* F);

/* sigma = argmax of the current fields (host [R][n]). */
fem_status fem_round(fem_solver* s, int32_t* sigma);
/* Integer evaluation of host configurations sigma [R][n]: value[B][R] is the
 * cut (MaxCut, bMinCut; each edge once) or the number of unsatisfied clauses
 * (Max-k-SAT); sizes[B][R][q] the group sizes for bMinCut, summed node weights
 * for a weighted problem (may be NULL).
 * Exact for integral weights (|total| < 2^53). */
fem_status fem_eval_int(const fem_problem* p, int32_t R, const int32_t* sigma, int64_t* value,
                        int64_t* sizes);
/* For callers that cannot allocate device memory (work recorded into a HIP
 * graph, tight serving loops, harnesses that forbid hipMalloc): the integer
 * evaluation of fem_eval_int on device-resident configurations, allocating
 * nothing.  Every intermediate (byte configurations, tile lists, per-tile
 * partial sums) lives in one fixed array of FEM_NOALLOC_SCRATCH_BYTES per
 * device, which the library holds from the first call on that device until
 * the process ends.  Results are bit-identical to fem_eval_int's.
 *  sigma: device int32 [R][n] (caller-owned, on the problem's device);
 *  value: device int64 [B][R]; sizes: device int64 [B][R][q] for bMinCut, or
 *    NULL (ignored for other kinds);
 *  hip_stream: the stream the work is enqueued on (NULL = the null stream).
 * The call only enqueues work: the outputs are valid once the stream has
 * reached that point.  A replica whose configuration holds a state outside
 * [0, q) gets value INT64_MIN and sizes -1 (the configuration is on the
 * device, so it is checked there, not on return).  Problems that would need
 * more than FEM_NOALLOC_SCRATCH_BYTES (about n*R bytes plus the partial sums)
 * give FEM_E_UNSUPPORTED with the size needed; NULL arguments or R < 1 give
 * FEM_E_INVAL.  All calls on one GPU share its array and keep no state in it
 * between calls: calls that overlap on one GPU (on different streams, or
 * from different threads, without ordering) race and give wrong results;
 * order them on one stream or synchronise in between. */
#define FEM_NOALLOC_SCRATCH_BYTES (64u << 20)
fem_status fem_eval_int_noalloc(const fem_problem* p, int32_t R, const int32_t* sigma, int64_t* value,
                                int64_t* sizes, void* hip_stream);
/* Round the current fields, evaluate, and return per instance the best
 * replica (max cut; min unsat; min 2*cut + lambda*sum_s |Pi_s|(|Pi_s|-1) for
 * bMinCut, 2*cut + lambda*(sum_s W_s^2 - sum_i V_i^2) with node weights;
 * ties to the lowest replica index), its value, and (if sigma is not
 * NULL) its configuration as int32 over all n nodes.  replica, value: [B]. */
fem_status fem_best(fem_solver* s, int32_t* replica, int64_t* value, int32_t* sigma);
/* Best value seen by the anytime read-out so far, [B][R] (eval_every > 0):
 * the cut (MaxCut; -inf before the first read-out), the number of unsatisfied
 * clauses (Max-k-SAT) or the integer energy 2*cut + lambda*sum_s
 * |Pi_s|(|Pi_s|-1) (bMinCut; with node weights as in fem_best); +inf before the first read-out otherwise. */
fem_status fem_anytime_best(fem_solver* s, double* value);

/* Checkpoint: bytes needed / write / restore (h, Adam moments, t).  Resuming
 * from a checkpoint reproduces an uninterrupted run bit for bit. */
fem_status fem_state_size(const fem_solver* s, size_t* bytes);
fem_status fem_get_state(fem_solver* s, void* buf, size_t bytes);
fem_status fem_set_state(fem_solver* s, const void* buf, size_t bytes);

/* --------------------------------------------------------------- tiling */
/* Launch shape of the step kernels.  vec: values per lane along the replica
 * axis (1, 2, 4, 8; Potts uses q); waves: wavefronts per workgroup (1..16,
 * fewer for register-heavy kernels); rows: rows per team per tile (1..64);
 * nt: 1 = non-temporal loads and stores of h and the Adam moments; lanes: cap
 * on the lanes of a team (0 = 64, else a power of two <= 64).  A team of L
 * lanes covers L*vec replicas of a row; where that is fewer than R the
 * replicas are split into segments and consecutive workgroups take different
 * segments of the same rows, so that each XCD (workgroups are dealt to the
 * eight XCDs round-robin) gathers from its own columns of the marginal copy.
 * fem_get_tile reports the lanes actually used.  All shapes give
 * bit-identical fields. */
typedef struct {
    int32_t vec, waves, rows, nt, lanes;
} fem_tile;
fem_status fem_get_tile(const fem_solver* s, fem_tile* t);
fem_status fem_set_tile(fem_solver* s, const fem_tile* t);
/* Autotune: time every valid shape twice for trial_steps steps from the same
 * state (restored afterwards), keep the shape with the fastest run, and cache it on disk under the key (kind, n,
 * nnz, R, q, dtype, instances, energies on/off, gradient mode) in
 * $FEM_TUNE_CACHE (default ~/.cache/femx/tune.txt).  use_cache = 1 returns a
 * cached choice without timing: the user's cache first, then the shapes
 * tuned on an MI355X that ship beside the library (data/tune_mi355x.txt). */
fem_status fem_tune(fem_solver* s, int32_t trial_steps, int32_t use_cache, fem_tile* chosen);

/* Average duration in milliseconds of the step kernel over the last
 * fem_step/fem_run call, measured with HIP events on the solver's stream
 * (0 if not measured).  Enabled by fem_profile(s, 1). */
fem_status fem_profile(fem_solver* s, int32_t on);
fem_status fem_profile_result(fem_solver* s, double* step_kernel_ms, int32_t* n_kernels);

/* ----------------------------------------------------- learned warm start */
/* A two-layer message-passing network (width 64) that maps the state of one
 * MaxCut replica part-way through an anneal to a proposal for that replica's
 * final read-out: one logit z_i per node, from which the anneal continues
 * with fields alpha * z and a shorter, colder schedule.  Trained on FEM's own
 * runs; an addition on top of the method (the paper has no network).
 * Node features from the replica's fields s: [1, ln(1+deg), mean incident
 * weight, tanh(s_i/2), clamp(s_i/4, -2, 2), three uniforms in [-1,1) from
 * Philox4x32-10 with counter (node, draw, 0, 0) and key (seed mod 2^32,
 * seed div 2^32)].  Layers: pre1 = x A1 + a(x) B1 + b1, H1 = relu(pre1);
 * pre2 = H1 A2 + a(H1) B2 + b2, H2 = relu(pre2); z = H2 c + d;
 * a(v)_i = sum_j W_ij v_j / max(deg_i, 1).  Weights are used as bfloat16 with
 * float32 arithmetic; the 9409 float32 master parameters are laid out
 * A1 [8][64], B1 [8][64], b1 [64], A2 [64][64], B2 [64][64], b2 [64], c [64],
 * d [1].  The network calls run on the null stream and return after their
 * work has finished. */
typedef struct fem_mpnn fem_mpnn;

/* theta0: 9409 host float32 initial parameters (n_params must be 9409). */
fem_status fem_mpnn_create(int device, const float* theta0, int32_t n_params, fem_mpnn** out);
void fem_mpnn_destroy(fem_mpnn* m);
/* master parameters (host, 9409 float32); set also resets the Adam moments. */
fem_status fem_mpnn_get_params(fem_mpnn* m, float* theta);
fem_status fem_mpnn_set_params(fem_mpnn* m, const float* theta);
/* logits z [n] of a MaxCut problem (or batch) for one replica's fields
 * state [n] and one feature draw; state and z are both host or both device. */
fem_status fem_mpnn_forward(fem_mpnn* m, const fem_problem* p, const float* state, uint64_t seed, int32_t draw,
                            float* z, int on_device);
/* One training step on a MaxCut batch (fem_batch_create, or one instance):
 * state [n] host float32, the fields of one replica of each instance at the
 * early step; labels [n] host int32 in {0, 1}, the final read-out of the same
 * replica; features of draw draw0; loss = mean over instances of BCE(z, y),
 * BCE = mean over the instance's nodes of softplus(z) - y z; the gradient is
 * taken wrt the bfloat16 weights and applied to the master weights by Adam
 * (0.9, 0.999, 1e-8, learning rate lr).  loss and grad_out (9409, host) may
 * be NULL. */
fem_status fem_mpnn_train_step(fem_mpnn* m, const fem_problem* batch, const float* state, const int32_t* labels,
                               uint64_t seed, int32_t draw0, double lr, double* loss, float* grad_out);
/* Proposal for R replicas: h_out[i][r] = alpha * z_i, z the logits of
 * replica r's fields state[i][r] with feature draw r; state and h_out are
 * [n][R] float32, both host or both device (they may not overlap).  All
 * replicas go through one pass: the graph inputs and their aggregates are
 * formed once, and layer 2 recomputes each neighbour's layer-1 activations
 * for 32 replicas at a time on the matrix cores, with the activations split
 * into three bfloat16 parts that sum to them exactly; the arithmetic is that
 * of float32 up to summation order (fem_mpnn_forward's per-replica pass can
 * differ from it by rounding).  Device work buffers of about 40 n R bytes are
 * kept between calls. */
fem_status fem_mpnn_infer(fem_mpnn* m, const fem_problem* p, int32_t R, const float* state, uint64_t seed,
                          float alpha, float* h_out, int on_device);
/* fem_mpnn_infer for device arrays, enqueued on the HIP stream `stream`
 * (NULL: the null stream) without waiting for it: the proposal is ready when
 * work queued after it on that stream runs, and execution errors show at the
 * caller's next synchronisation.  The work buffers belong to the network
 * object, so calls on one object must be ordered (one stream, or events);
 * calls that overlap on different streams race.  A call that has to grow
 * the buffers frees the old ones, which waits for the device. */
fem_status fem_mpnn_infer_async(fem_mpnn* m, const fem_problem* p, int32_t R, const float* state, uint64_t seed,
                                float alpha, float* h_out, void* stream);
/* parameter file: 8-byte magic "FEMMPNN1", int32 9409, 9409 float32. */
fem_status fem_mpnn_save(fem_mpnn* m, const char* path);
fem_status fem_mpnn_load(fem_mpnn* m, const char* path);

#ifdef __cplusplus
}
#endif
#endif /* FEM_H */
