/*
 * bbp.h -- C ABI of the MI355X blockBP surface-code decoder.
 *
 * The decoder is the blockBP decoder of Kaufmann & Arad, "A blockBP decoder for the surface code"
 * (arXiv 2402.04834): for every syndrome it builds the tensor network of each of the four logical
 * cosets (Sec. III.A), partitions it into rectangular blocks, runs belief propagation between blocks
 * with boundary-MPS messages of bond dimension at most chi (Sec. III.D), estimates every coset
 * probability with the Bethe formula of Lemma 3.1 and returns the most likely coset (Alg. 1).
 *
 * Conventions shared by every entry point:
 *   grid of L = 2d-1 rows and columns; qubits at (r+c) even, numbered row-major; Z-checks (site
 *   operators A_u) at (even r, odd c), X-checks (plaquettes B_p) at (odd r, even c); a syndrome is m =
 *   2d(d-1) bytes (0/1), Z-checks row-major then X-checks row-major; a single-qubit Pauli is coded
 *   x + 2z (0 = I, 1 = X, 2 = Z, 3 = Y); coset index 0..3 = I, X, Y, Z where X is X on row 0 of
 *   horizontal edges and Z is Z on column 0 of horizontal edges.
 *
 * Errors: every int-returning function returns BBP_OK (0) or a negative code; bbp_last_error() gives a
 * message for the calling thread's last failure. No C++ exception crosses this boundary. A coset whose
 * BP loop did not converge is not an error: it is reported through delta/iters and the decision rule.
 */
#ifndef BBP_H
#define BBP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BBP_OK 0
#define BBP_EINVAL (-1)        /* an argument is out of range or inconsistent */
#define BBP_ENOMEM (-2)        /* a host or device allocation failed */
#define BBP_EHIP (-3)          /* a HIP runtime call failed (message carries the HIP error string) */
#define BBP_EUNSUPPORTED (-4)  /* valid options outside what the GPU path implements */

/* Decoder parameters (Sec. III.E, "Decoder Parameters"; run values of Sec. IV). */
typedef struct bbp_opts {
  int32_t block_rows;   /* block height k_r in tensors (remark 1: edge blocks hold the remainder) */
  int32_t block_cols;   /* block width k_c */
  int32_t chi;          /* maximal MPS bond dimension of messages and of the in-block boundary MPS */
  int32_t max_iter;     /* BP iterations; one iteration = both colour rounds (remark 8) */
  double delta0;        /* exit threshold on the convergence distance (remark 4) */
  double delta1;        /* trust threshold of the decision rule (remark 6); delta0 <= delta1 */
  double damping;       /* eta of remark 7: m <- (1-eta) m_new + eta m_old; 0 <= eta < 1 */
  int32_t rule;         /* 0 = rule of Alg. 1 / remark 6, 1 = plain argmax of the Bethe estimates */
  int32_t fixed_iters;  /* 1 = always run max_iter iterations (no early exit) */
  int32_t precision;    /* 0 = FP32 block contractions; 1 = the contractions with the side messages' middle sites
                           that run on the matrix cores (sweeps of 5 and 6 steps) take BF16 operands with FP32
                           accumulation, the qubit tensor of an adjacent end site folded into the message operand;
                           every other product stays FP32. Both: FP64 convergence distance and Bethe sums */
  int32_t graph;        /* 1 = capture the decode of a call into a HIP graph on first use and replay it on
                           later calls with identical arguments (pointers, sizes, options, stream); needs a
                           stream other than the default stream; ignored when timing is requested. At most
                           64 graphs are kept; the 65th argument set empties the cache (after a device
                           synchronisation) */
  double gate;          /* 0 = the paper's schedule. > 0: residual-gated schedule, a scheduling variant (Sec. IV
                           leaves smarter scheduling open): in a colour round the update of message u->v is
                           skipped for a coset when u->v itself and every message entering block u other than
                           v->u changed, in their most recent updates, by a distance term 2 - 2<m, m_old>^2
                           below gate; a skipped message keeps its value and its term becomes 0 (so it also
                           counts 0 in Delta) */
} bbp_opts;

/* Defaults of Sec. IV: 6x6 blocks, chi 16, 20 iterations, delta0 1e-4, delta1 1e-2, eta 0.1; eager
 * launches (graph 0). */
void bbp_default_opts(bbp_opts* opts);

/* Message for the calling thread's most recent non-zero return; never NULL. */
const char* bbp_last_error(void);

/* ---------------------------------------------------------------------------------------------------
 * Host-side network (Alg. 1, first steps): f_s, the four coset labels f_s L, and the block plan.
 * `syndrome` is a host array of m = 2d(d-1) bytes (0/1). The network is owned by the caller after a
 * successful return and must be released with bbp_free_network. Errors: BBP_EINVAL for d < 2,
 * m != 2d(d-1), p outside (0, 1) or a byte other than 0/1; BBP_ENOMEM.
 */
typedef struct bbp_net bbp_net;
int bbp_build_network(int32_t d, double p, const uint8_t* syndrome, int64_t m, bbp_net** out);
/* d, number of qubits n and of checks m of a network. */
int bbp_net_dims(const bbp_net* net, int32_t* d, int32_t* n, int32_t* m);
/* Coset labels of the network: labels[4][L*L] (host), bit 0 = x and bit 1 = z of f_s L at every grid
 * site, row-major (check sites hold 0). */
int bbp_net_labels(const bbp_net* net, uint8_t* labels);
void bbp_free_network(bbp_net* net);

/* ---------------------------------------------------------------------------------------------------
 * Plan summary for distance d under `opts` (Sec. III.D-E): block grid, number M of directed messages
 * per coset, and the result of the plan-time rank analysis. `exact_sweeps` is 1 when no boundary MPS
 * inside any block update can exceed bond chi for any input, so that truncation is the identity and the
 * GPU contracts blocks exactly; `flops_per_iter` / `flops_bethe` are the algorithmic FP32 flops of one
 * coset-iteration / of the Bethe sweeps of one coset: the multiply-adds (2 flops each) of the block
 * contractions -- qubit tensors against their partner configuration and the emitted side-message bonds
 * they use, and the contractions with the dense middle site of every side message; COPY tensors and the
 * side-message sites that only route a bond count zero -- plus 10 flops per configuration for the closing
 * normalisation, damping and distance term. Errors: BBP_EINVAL for invalid opts.
 */
typedef struct bbp_plan_info {
  int32_t L, n, m;
  int32_t block_grid_rows, block_grid_cols;
  int32_t num_messages;          /* M */
  int32_t updates_per_iter;      /* = M */
  int32_t exact_sweeps;          /* 1: chi never truncates (see above) */
  int32_t max_cut_rank;          /* largest generic Schmidt rank among the cuts whose dimensions exceed chi on
                                    both sides -- the only cuts where truncation to chi could act; 0 if none.
                                    At or below chi it means truncation never acts (exact_sweeps = 1) */
  int32_t gpu_supported;         /* 1: bbp_decode_device accepts these options */
  double flops_per_iter;
  double flops_bethe;
  int32_t truncating_sweeps;     /* sweeps (BP rounds and closing) that run in the truncating kernel: those whose
                                    boundary MPS can exceed chi, and every sweep of a plan with blocks wider than
                                    6; their flops count QR, reflection and SVD work (see below) */
  int32_t message_stride;        /* S: floats per stored dense message, 2^max(6, widest block); the message
                                    arrays of bbp_decode_device and bbp_group are [batch][4][M][S] */
} bbp_plan_info;
int bbp_plan_query(int32_t d, const bbp_opts* opts, bbp_plan_info* info);

/* ---------------------------------------------------------------------------------------------------
 * Device workspace needed by bbp_decode_device for `batch` syndromes of distance d (bytes, 256-byte
 * aligned sub-buffers). A plan with truncating sweeps adds one 273 KB FP64 slot per truncating sweep of a
 * colour round and coset job, at most 32768 slots (8.9 GB; larger rounds run in chunks of that many).
 * Errors: BBP_EINVAL.
 */
int bbp_workspace_size(int32_t d, int64_t batch, const bbp_opts* opts, size_t* bytes);

/* Optional per-call timing of the kernels (filled when non-NULL; adds one event pair per launch and a
 * stream synchronisation at the end of the call). */
typedef struct bbp_timing {
  double update_ms;          /* summed duration of the block-sweep launches of the BP rounds */
  int32_t update_launches;   /* one launch per sweep class per colour round */
  double bethe_ms;           /* closing sweeps of the Bethe estimate */
  double other_ms;           /* labels, init, convergence, decision */
  double update_flops;       /* algorithmic flops of the update launches actually executed */
  /* The sweep-kernel instantiation with the largest summed duration in the BP rounds. Its class code is
   * (((steps - 1) * 4 + top * 2 + bottom) * 2 + single) * 2 + q00: sweep length 1..6, side messages
   * present at the top / bottom end of the columns, one position across the sweep, first site a qubit. */
  int32_t top_class;
  int32_t top_launches;
  double top_ms;
  double top_flops;
} bbp_timing;

/* ---------------------------------------------------------------------------------------------------
 * Whole decoder (Alg. 1) on a batch of syndromes resident in device memory.
 *   syndromes_dev   [batch][m] uint8 (0/1), device
 *   workspace       device buffer of at least bbp_workspace_size bytes, owned by the caller
 *   loglik_dev      [batch][4] float64, device: Bethe estimate ln Z of each coset (order I, X, Y, Z);
 *                   NaN when a closing contraction or edge overlap was not positive
 *   delta_dev       [batch][4] float64: final convergence distance (+inf for such untrusted cosets)
 *   iters_dev       [batch][4] int32: BP iterations run
 *   coset_dev       [batch] uint8: decided coset
 *   correction_dev  [batch][n] uint8: codes x + 2z of the correction f_s L*
 *   messages_dev    optional [batch][4][M][S] float32: final dense messages (unit norm; entry index
 *                   = crossing-bond values, first site most significant; S = message_stride of
 *                   bbp_plan_query, 64 unless a block is wider than 6); NULL to skip
 *   stream          hipStream_t on which all work is enqueued (NULL = default stream); the call
 *                   returns after enqueueing unless `timing` is non-NULL.
 * All pointers are caller-owned; nothing is allocated per call (plans are cached per (d, opts) on first
 * use). Block sweeps whose boundary MPS can exceed chi (and every sweep of a plan with blocks wider than 6)
 * run the boundary-MPS compression of Sec. III.D on the device: a Householder QR sweep and a truncated
 * one-sided Jacobi SVD sweep after every column, in FP64, with each side message entering with its
 * not-yet-absorbed part an isometry; the others contract exactly. Errors: BBP_EINVAL (bad sizes, NULL required
 * pointer, workspace too small), BBP_EUNSUPPORTED (blocks wider than 8; chi below 2^(k/2), which would
 * truncate the messages themselves; chi above 16 where a sweep needs the truncating kernel), BBP_EHIP.
 */
int bbp_decode_device(int32_t d, double p, const uint8_t* syndromes_dev, int64_t batch,
                      const bbp_opts* opts, void* workspace, size_t workspace_bytes,
                      double* loglik_dev, double* delta_dev, int32_t* iters_dev, uint8_t* coset_dev,
                      uint8_t* correction_dev, float* messages_dev, void* stream, bbp_timing* timing);

/* ---------------------------------------------------------------------------------------------------
 * Allocation-free decode, for callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc. Same semantics and results as bbp_decode_device
 * (the same kernels, eager launches on `stream`, one stream, no timing, no message output), but the
 * workspace and the plan's device tables live in a static device array of BBP_SCRATCH_BYTES that the
 * library holds on every device it runs on until the process ends; the call itself allocates nothing (no
 * hipMalloc, no hipFree, no allocating library routine) and enqueues the upload of the plan tables from
 * host memory that the library keeps for the life of the process. The caller owns syndromes and outputs
 * (device pointers, layouts as bbp_decode_device).
 * Limit: the plan tables plus bbp_workspace_size(d, batch, opts) must fit in BBP_SCRATCH_BYTES;
 * bbp_noalloc_max_batch gives the largest batch that fits (about 500 syndromes at d=17 with 6x6 blocks).
 * Every call on a device shares that device's array, which keeps the last call's contents (nothing in it
 * needs to start at zero: the decode writes every entry it reads): calls that overlap on one device race,
 * so a caller serialises them (one stream, or events).
 * Errors: BBP_EINVAL (arguments as bbp_decode_device; a batch beyond the limit, with the bytes it needs),
 * BBP_EUNSUPPORTED, BBP_EHIP.
 */
#define BBP_SCRATCH_BYTES (64u << 20)
int bbp_decode_device_noalloc(int32_t d, double p, const uint8_t* syndromes_dev, int64_t batch,
                              const bbp_opts* opts, double* loglik_dev, double* delta_dev, int32_t* iters_dev,
                              uint8_t* coset_dev, uint8_t* correction_dev, void* stream);
int bbp_noalloc_max_batch(int32_t d, const bbp_opts* opts, int64_t* max_batch);

/* ---------------------------------------------------------------------------------------------------
 * Mixed batches. A group is a batch of syndromes of one distance d (and bond dimension chi), each with its
 * noise rate p, resident in device memory, with the device arrays that receive its results (layouts as in
 * bbp_decode_device). One call
 * decodes up to 8 groups together: every colour round launches each block-sweep class once over all
 * groups, so a mix of distances costs no more launches than its largest member.
 */
typedef struct bbp_group {
  int32_t d;
  int32_t chi;                    /* this group's bond dimension chi; 0 = opts->chi */
  double p;                       /* noise rate of every syndrome of the group, unless p_dev is given */
  const double* p_dev;            /* optional [batch] device array: each syndrome's own p in (0, 1) */
  const uint8_t* syndromes_dev;   /* [batch][2d(d-1)] */
  int64_t batch;
  double* loglik_dev;             /* [batch][4] */
  double* delta_dev;              /* [batch][4] */
  int32_t* iters_dev;             /* [batch][4] */
  uint8_t* coset_dev;             /* [batch] */
  uint8_t* correction_dev;        /* [batch][d^2 + (d-1)^2] */
  const float* init_messages_dev; /* optional [batch][4][M][S] start messages (dense, layout of messages_dev of
                                     bbp_decode_device), each scaled to unit norm by the decoder, entries beyond
                                     2^K ignored, an all-zero or non-finite one replaced by the uniform start;
                                     NULL = the uniform start of remark 2 */
  float* messages_dev;            /* optional [batch][4][M][S] output: final messages, as in bbp_decode_device */
  double noise[4];                /* optional biased Pauli noise: probabilities of I, X, Z, Y (index = code x + 2z),
                                     non-negative, summing to 1, noise[0] > 0; all zero = depolarizing with p.
                                     Exclusive with p_dev; opts->precision 0 only (else BBP_EUNSUPPORTED). */
} bbp_group;

/* Workspace for bbp_decode_groups (the groups' own workspaces laid end to end). Output and syndrome
 * pointers are not read. Errors: BBP_EINVAL (ngroups outside [1, 8], invalid d, p, batch or opts). */
int bbp_workspace_size_groups(const bbp_group* groups, int32_t ngroups, const bbp_opts* opts, size_t* bytes);

/* Whole decoder (Alg. 1) on the groups, with the semantics of bbp_decode_device per group (results are
 * identical to decoding each group alone). Errors as bbp_decode_device. */
/* The launch variant of a call is the one tuned (bbp_autotune / bbp_set_tuning) for the group with the most
 * work (syndromes x flops per iteration), else the default. */
int bbp_decode_groups(const bbp_group* groups, int32_t ngroups, const bbp_opts* opts, void* workspace,
                      size_t workspace_bytes, void* stream, bbp_timing* timing);

/* ---------------------------------------------------------------------------------------------------
 * Launch tuning. The block sweeps of a round can be enqueued with the items of a launch in sweep-major
 * or job-major order, and spread over 1, 2 or 4 streams (a round's launches are independent). Results do
 * not depend on the choice. bbp_autotune times every variant on the given batch (a warm-up and two
 * timed decodes each, on `stream`; it allocates and frees a small device output buffer), keeps the
 * fastest for (d, block size, chi) on the current device, and returns it; later decodes of that key use
 * it. bbp_set_tuning sets it directly. Errors: BBP_EINVAL, BBP_ENOMEM, BBP_EHIP. */
typedef struct bbp_tuning {
  int32_t order;     /* 0 sweep-major, 1 job-major */
  int32_t streams;   /* 1, 2 or 4 */
  double ms;         /* decode time of the chosen variant on the tuning batch (output of bbp_autotune) */
} bbp_tuning;
int bbp_autotune(int32_t d, double p, const uint8_t* syndromes_dev, int64_t batch, const bbp_opts* opts,
                 void* workspace, size_t workspace_bytes, void* stream, bbp_tuning* best);
int bbp_set_tuning(int32_t d, const bbp_opts* opts, const bbp_tuning* tuning);

/* Host convenience: decode host-side networks (up to 8 distinct (d, p) in one call, in any order) and
 * return host outputs in input order with the layouts of bbp_decode_device; correction rows are n_max
 * bytes, n_max the largest qubit count in the call, the first n(d) of each row used and the rest 0.
 * Allocates and frees its own device memory and synchronises. Errors as above. */
int bbp_blockbp_decode(bbp_net* const* nets, int64_t batch, const bbp_opts* opts, double* loglik,
                       double* delta, int32_t* iters, uint8_t* coset, uint8_t* correction);

/* ---------------------------------------------------------------------------------------------------
 * Boundary-MPS decoder: the single-block limit of blockBP (Sec. III.D), i.e. the bMPS decoder of Sec.
 * III.A that Sec. IV runs with chi = 16 as its accuracy reference. Each coset network is contracted column
 * by column, left to right, as an MPS over the L rows; after every column but the last the MPS is
 * compressed to bond dimension chi (a QR sweep from the top row down, then a truncated-SVD sweep from the
 * bottom row up keeping the chi largest singular values of every bond, the norm split off into an FP64
 * log-scale); the last column's chain of matrices is multiplied out. One wavefront per coset network;
 * matrix work in FP64 (an estimate is resolved down to about the unit roundoff times the state's norm, which
 * the likeliest configurations set, so FP32 would leave cosets some tens of nats below the best unresolved).
 *
 * Workspace: bbp_bmps_workspace_size bytes (coset labels plus 16*2*16 + 32*64 + 32 doubles per grid row and
 * coset network -- the compressed row and its factor in compact form: about 20.3 KiB * L * 4 * batch). Errors: BBP_EINVAL (d outside [2, 32], chi outside [1, 16], batch < 0
 * or above 2^22).
 */
int bbp_bmps_workspace_size(int32_t d, int64_t batch, int32_t chi, size_t* bytes);

/* Decode `batch` syndromes resident in device memory (uint8 [batch][2d(d-1)]), enqueued on `stream` (a
 * hipStream_t; NULL = the default stream).
 *   noise: p in (0, 1) (depolarizing) unless p_dev ([batch] device doubles, each syndrome's own p) or
 *          noise (host double[4]: Pauli probabilities of I, X, Z, Y by code x + 2z, summing to 1, noise[0]
 *          > 0; exclusive with p_dev) is given;
 *   loglik_dev [batch][4]: the estimates of ln pi(f_s L G), L in (I, X, Y, Z), NaN where the contraction
 *          ended with a value that is not positive;
 *   coset_dev [batch]: the largest estimate (NaN as -inf, ties to the lowest index);
 *   correction_dev [batch][n] (may be NULL): f_s L* as Pauli codes x + 2z;
 *   kernel_ms (host, may be NULL): duration of the contraction kernel, measured with HIP events on the
 *          stream (the call then synchronises with the stream).
 * batch 0 is a no-op. Errors: BBP_EINVAL (arguments, workspace too small), BBP_EHIP. */
int bbp_bmps_decode_device(int32_t d, double p, const double* p_dev, const double* noise,
                           const uint8_t* syndromes_dev, int64_t batch, int32_t chi, void* workspace,
                           size_t workspace_bytes, double* loglik_dev, uint8_t* coset_dev, uint8_t* correction_dev,
                           void* stream, float* kernel_ms);

/* ---------------------------------------------------------------------------------------------------
 * Learned warm start. BP of blockBP starts from uniform messages (remark 2); the paper names machine
 * learning as a way to improve BP (Sec. V, summary and conclusions). Here a convolutional network
 * predicts the start messages of every coset job from the local syndrome, and the decoder runs from them.
 *
 * Network (per coset job, on the L x L grid): 11 input channels per site (x and z bits of the coset label
 * f_s L at qubits, the syndrome bit at checks, qubit / Z-check / X-check indicators, p, 1, the coset's x and
 * z bits, at checks the generator bit G), where G is the prefix parity of f_s L on the horizontal edges
 * above a plaquette in its column (x part) or left of a vertex in its row (z part); three 3x3 convolutions
 * with zero padding (11 -> 64 -> 128 -> 96 channels, ReLU after the first two) give features
 * F; for each directed message with K legs (leg i joins site a_i of the sending block to site b_i across the
 * boundary, leg 0 at the top / left) and f_i = [F(a_i), F(b_i)], the weights of the message's direction
 * (E, W, S, N) give u_i = Wu^T f_i + bu (2 values) and P_i = Wp^T [f_i, f_{i+1}] + bp (4 values); the
 * message is exp(s) scaled to unit norm, s(b) = sum_i u_i[b_i] + sum_i P_i[2 b_i + b_{i+1}] over the 2^K
 * leg configurations b (leg 0 the most significant bit, the layout of the decoder's messages).
 * Parameters: one float32 device array of bbp_warm_param_count() values, in the order conv1 W [99][64],
 * b [64], conv2 W [576][128], b [128], conv3 W [1152][96], b [96], then for E, W, S, N: Wu [192][2], bu [2],
 * Wp [384][4], bp [4]; W rows are (3 dy + dx) * C_in + c_in for the input site (r + dy - 1, c + dx - 1).
 * Training loss of a message against a converged cold-start message t (non-negative): KL(q || p) of
 * q = t / sum(t) and p = softmax(s).
 * All pointers are device pointers unless stated; work is enqueued on `stream` (NULL = default stream).
 * Errors: BBP_EINVAL (range, NULL, workspace too small), BBP_EUNSUPPORTED (blocks larger than 6),
 * BBP_EHIP; bbp_warm_last_error() gives the message. */
const char* bbp_warm_last_error(void);
int bbp_warm_param_count(int64_t* count);

/* Workspace of bbp_warm_predict (train = 0; bounded: the forward runs in chunks of 512 syndromes) or of
 * bbp_warm_loss_grad (train = 1; grows with batch). */
int bbp_warm_workspace_size(int32_t d, int64_t batch, const bbp_opts* opts, int32_t train, size_t* bytes);

/* Predicted start messages of batch syndromes [batch][2d(d-1)] (noise rate p, or p_dev [batch] when not
 * NULL): messages_dev [batch][4][M][64], unit norm, zero beyond 2^K (M and K as in bbp_plan_query).
 * precision 0: FP32 convolutions (the arithmetic of training); 1: BF16 weights and activations with FP32
 * accumulation (inference; the convolution weights are rounded to BF16 from params_dev on each call). */
int bbp_warm_predict(int32_t d, double p, const double* p_dev, const uint8_t* syndromes_dev, int64_t batch,
                     const bbp_opts* opts, const float* params_dev, int32_t precision, float* messages_dev,
                     void* workspace, size_t workspace_bytes, void* stream);

/* Loss and gradient of the network on a training batch: targets_dev [batch][4][M][64] (converged messages,
 * non-negative, entries beyond 2^K ignored), use_dev [batch * 4] (1 = train on every message of that coset
 * job), trained_messages = M times the number of used jobs. loss_dev[0] = sum over used messages of
 * KL(q || p) / trained_messages; grad_dev (param_count floats) receives its gradient (overwritten). */
int bbp_warm_loss_grad(int32_t d, double p, const double* p_dev, const uint8_t* syndromes_dev, int64_t batch,
                       const bbp_opts* opts, const float* params_dev, const float* targets_dev,
                       const uint8_t* use_dev, int64_t trained_messages, float* grad_dev, float* loss_dev,
                       void* workspace, size_t workspace_bytes, void* stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected with step >= 1) on the parameters; m_dev
 * and v_dev are the moment arrays (param_count floats each, zero before step 1). */
int bbp_warm_adam(float* params_dev, const float* grad_dev, float* m_dev, float* v_dev, int64_t step, float lr,
                  void* stream);

/* Warm-started decode with cold fallback: the network's messages start BP (bbp_group.init_messages_dev);
 * every syndrome with a coset whose final distance is not below opts->delta1, or whose decided coset took
 * more iterations than another of its cosets (the right coset converges fastest, Sec. IV), is decoded again
 * from the uniform start, and its results replace the warm ones (its iteration counts are the sum of both
 * runs). [trained_d_min, trained_d_max] are the distances the parameters were trained on (both 0: no range):
 * for d outside them the whole batch is decoded from the uniform start and *fallback_count = batch, because
 * there the predicted starts lead BP to other fixed points that pass every convergence test. Outputs as
 * bbp_decode_device; *fallback_count (host, may be NULL) receives the number of syndromes decoded from the
 * uniform start. The call synchronises `stream` once (to size the fallback batch). precision: the network's,
 * as bbp_warm_predict. Errors as bbp_warm_predict, BBP_EINVAL for a range with min > max or one bound 0. */
int bbp_warm_decode_workspace_size(int32_t d, int64_t batch, const bbp_opts* opts, size_t* bytes);
int bbp_warm_decode(int32_t d, double p, const double* p_dev, const uint8_t* syndromes_dev, int64_t batch,
                    const bbp_opts* opts, const float* params_dev, int32_t precision, int32_t trained_d_min,
                    int32_t trained_d_max, void* workspace, size_t workspace_bytes,
                    double* loglik_dev, double* delta_dev, int32_t* iters_dev, uint8_t* coset_dev,
                    uint8_t* correction_dev, int64_t* fallback_count, void* stream);

/* ---------------------------------------------------------------------------------------------------
 * Validation hook (host, float64): evaluates the block message update that produces message `msg_id`
 * (or, with msg_id = -1 - b, the closing sweep of block b) with exactly the index arithmetic of the GPU
 * kernel, for one coset. `labels` is the L*L label grid of that coset (bit 0 = x, bit 1 = z), `msgs` the
 * current dense messages [M][64] (host), `out` receives the 2^kp-entry unnormalised outgoing state scaled
 * to unit norm and `logscale` the natural log of the scale split off during the sweep. Used by the CPU
 * test-suite to check the plan against the oracle; no decode path calls it.
 * Errors: BBP_EINVAL for an unknown id or NULL pointers. */
int bbp_reference_update_host(int32_t d, double p, const bbp_opts* opts, const uint8_t* labels, int32_t msg_id,
                              const double* msgs, double* out, double* logscale);

#ifdef __cplusplus
}
#endif

#endif /* BBP_H */
