/*
 * sdnn.h -- C ABI of the MI355X (gfx950) layered sparse-DNN library.
 *
 * The library runs the computation that dominates the paper's large sparse
 * neural-network workload (section "Large Sparse Neural Network Inference"):
 * inference of a stack of L sparse layers over a batch of input rows,
 *
 *     Y_{l+1} = min(c, max(0, Y_l W_l + b_l)),      l = 0 .. L-1,   c = 32,
 *
 * where every output neuron j of W_l has exactly k = 32 input neurons.  The
 * paper checks the result against "truth categories"; here the equivalent
 * output is the ascending list of rows whose final activations are nonzero.
 * The paper issues the GPU work of that workload as task graphs (section
 * "Heterogeneous Tasking", the cudaFlow; section "Scheduling GPU Tasks", one
 * graph per cudaFlow submitted in a single call); the forward pass here can run
 * as one hipGraph of per-layer kernels, as one
 * persistent cooperative kernel, or as eager launches (sdnn_set_exec).
 * A backward pass (gradients of W values on the fixed pattern, of b and of Y_0)
 * with layer checkpointing is provided for training.
 *
 * Conventions for every entry point:
 *  - All pointers named "dev" are HIP device pointers; "host" pointers are host
 *    memory.  The caller allocates every buffer (the library allocates nothing
 *    on the device except hipGraph objects); the library never frees them.
 *  - Row-major fp32 activations: row r of a [rows][N] matrix starts at r*N.
 *  - Layer tensors are stacked: idx/w are [L][N][k] (neuron-major: slot s of
 *    neuron j of layer l at (l*N + j)*k + s), bias is [L][N].  Each neuron's
 *    k input ids must be distinct and ascending, in [0, N).
 *  - "stream" is a hipStream_t passed as void* (NULL = the default stream).
 *    Compute entry points only enqueue work and never synchronize the host;
 *    argument errors are reported synchronously and launch nothing.
 *  - Every function returns an sdnn_status; sdnn_last_error() gives a
 *    thread-local message for the last failure on the calling thread.
 *  - Concurrent calls on one sdnn_net must be serialized by the caller (they
 *    share the workspace).
 */
#ifndef SDNN_H
#define SDNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sdnn_net_s *sdnn_net;

typedef enum {
    SDNN_OK = 0,
    SDNN_EINVAL = -1,        /* bad argument; nothing was launched */
    SDNN_ENOMEM = -2,        /* workspace / checkpoint buffer too small */
    SDNN_EHIP = -3,          /* a HIP runtime call failed */
    SDNN_EUNSUPPORTED = -4,  /* valid request the library does not implement (e.g. k != 32) */
    SDNN_EDEVICE = -5        /* a kernel reported an error (barrier time-out, bad batch offsets) */
} sdnn_status;

/* sdnn_desc.flags */
#define SDNN_TRAINABLE     0x1u  /* build the transposed pattern; enables sdnn_backward */
#define SDNN_NO_COMPACTION 0x2u  /* process every row in every layer (results are identical) */
#define SDNN_DEBUG_CHECKS  0x4u  /* validate idx/w/bias on the device at create time (synchronizes) */
#define SDNN_AUTOTUNE      0x8u  /* time the kernel variants at create time and keep the fastest */
#define SDNN_NO_SCHEDULE   0x10u /* build no create-time slot schedules: the streamed-weight kernels
                                    read idx and w on every call, so the borrowed parameters (ids
                                    included) may change between calls, e.g. when layers are
                                    streamed through device slots */

/* sdnn_set_exec modes */
#define SDNN_EXEC_AUTO         0 /* GRAPH for one batch, GRAPH_MERGED for several; PERSISTENT
                                    on the wide-layer and chunked one-row-tile kernels (plan
                                    variants 3, 6 and 7) */
#define SDNN_EXEC_EAGER        1 /* one kernel launch per layer, batches one after another */
#define SDNN_EXEC_GRAPH        2 /* one hipGraph; batches one after another ("plain" form) */
#define SDNN_EXEC_PERSISTENT   3 /* all layers of all batches in one cooperative kernel ("batched") */
#define SDNN_EXEC_GRAPH_MERGED 4 /* one hipGraph whose layer nodes serve all batches ("batched") */

typedef struct {
    int32_t n_neurons;   /* N >= 1 (N <= 2^20) */
    int32_t n_layers;    /* L >= 1 */
    int32_t k;           /* inputs per neuron; must be 32 (else SDNN_EUNSUPPORTED) */
    float clamp;         /* c > 0 (32 for the challenge networks) */
    int32_t ckpt_every;  /* backward checkpoint stride S (>= 1) when SDNN_TRAINABLE, else 0 */
    uint32_t flags;      /* SDNN_* flags above */
    int64_t max_rows;    /* largest `rows` any later call will pass (workspace capacity) */
} sdnn_desc;

/* The tile plan of the forward layer kernel (chosen by heuristic or autotuner). */
typedef struct {
    int32_t rows_per_tile;   /* T: activation rows staged per workgroup tile */
    int32_t threads;         /* workgroup size */
    int32_t grid;            /* workgroups per layer launch (grid-stride over tiles) */
    int32_t variant;         /* 2 = scheduled resident-weight kernel, 0 = LDS-staged rows,
                                4 = one-row tiles with resident weights (forward-only nets of
                                    2048 < N <= 16384 neurons, N % 4 == 0), ascending slot order,
                                5 = the same with each neuron's slots in a create-time order
                                    that spreads a half-wave's LDS reads over distinct banks,
                                6 = one-row tiles staged in rows_per_tile = 2 or 4 chunks,
                                    resident weights of create-time neuron pairs (forward-only
                                    nets of 16384 < N <= 65536 neurons, N % 2048 == 0), each
                                    chunk's slots in a create-time bank-spreading order,
                                7 = the same images, two parts of 2048 neurons per workgroup
                                    (nets of variant 6 whose every layer has a single weight
                                    value, N % 4096 == 0; the default there; outputs equal
                                    variant 6's),
                                1 = direct gather (rows too wide for LDS),
                                3 = wide layers: rows packed T per tile [N][T] in the workspace,
                                    one T*4-byte gather per slot (forward-only nets whose
                                    shape the scheduled kernel cannot take) */
    float tuned_us;          /* measured time per full-live layer of the tuning shape (0 if untuned) */
} sdnn_plan;

/* Bytes of device workspace sdnn_create needs for this descriptor.
 * Paper: section "Large Sparse Neural Network Inference" (the net and the input
 * batches live on the GPU; the paper streams them through 8 GB GPUs, here they are
 * resident). */
sdnn_status sdnn_workspace_size(const sdnn_desc *desc, size_t *bytes);

/* Bytes of the checkpoint buffer a forward over `rows` rows must be given so that
 * sdnn_backward can run from it: (ceil(L / S) - 1) * rows * N * 4.
 * Paper: none (training is an extension of the layer rule of section "Large
 * Sparse Neural Network Inference"). */
sdnn_status sdnn_ckpt_size(const sdnn_desc *desc, int64_t rows, size_t *bytes);

/*
 * Create a network over caller-owned parameters.
 *   idx  dev int32 [L][N][k], w dev fp32 [L][N][k], bias dev fp32 [L][N].
 *   These are BORROWED: they must stay alive and keep their pattern until
 *   sdnn_destroy.  w and bias may be updated in place between calls (training).
 *   workspace: dev buffer of at least sdnn_workspace_size bytes, 256-B aligned,
 *   owned by the caller, used exclusively by this net until sdnn_destroy.
 * If any bias is > 0, an all-zero row no longer stays all-zero, so compaction and
 * early exit are switched off for the whole net (results are unchanged).
 * Synchronizes `stream` (create is not a timed path).
 * Paper: section "Large Sparse Neural Network Inference" (the problem's inputs:
 * L sparse layer matrices and their biases) and section "Heterogeneous Tasking"
 * (a GPU task graph is built once, then offloaded).
 */
sdnn_status sdnn_create(const sdnn_desc *desc, const int32_t *idx, const float *w, const float *bias,
                        void *workspace, size_t ws_bytes, void *stream, sdnn_net *out);

/* Choose how sdnn_forward runs the layer chain (SDNN_EXEC_*).
 * Paper: section "Scheduling GPU Tasks" (one GPU task graph launched in one call)
 * and the graph-construction comparison of section "Large Sparse Neural Network
 * Inference". */
sdnn_status sdnn_set_exec(sdnn_net net, int32_t mode);

/* Read the current tile plan.  Paper: none (the GPU kernel's shape is left open
 * in section "Large Sparse Neural Network Inference"). */
sdnn_status sdnn_get_plan(sdnn_net net, sdnn_plan *plan);

/* Select the kernel variant given by plan->rows_per_tile, plan->threads and
 * plan->variant (plan->grid and plan->tuned_us are ignored; the grid follows from
 * the variant's occupancy).  SDNN_EINVAL if no variant has those three values,
 * SDNN_EUNSUPPORTED if it does not fit this net (LDS, schedule, workspace).  Variants
 * of one family (0, 1 and 3; or 2) give bitwise-equal results.  Not thread-safe
 * against calls on the same net.  Paper: none (as sdnn_get_plan). */
sdnn_status sdnn_set_plan(sdnn_net net, const sdnn_plan *plan);

/*
 * Kernel timing (measurement support, not part of the method).  With enable != 0,
 * every sdnn_forward in SDNN_EXEC_PERSISTENT mode records a pair of HIP events
 * around its persistent layer-chain kernel, on the stream it is launched on.
 * sdnn_kernel_time waits for the recorded events and returns the summed kernel
 * time in milliseconds and the number of launches since the previous call (or
 * since timing was enabled), then starts a new sum.  Either output pointer may
 * be NULL.  Events are created on first use and released by sdnn_destroy.
 * Paper: none (measurement support).
 */
sdnn_status sdnn_set_timing(sdnn_net net, int32_t enable);
sdnn_status sdnn_kernel_time(sdnn_net net, double *total_ms, int32_t *launches);

/* Autotuner of the layer kernel's tile plan (rows per tile, workgroup size, kernel
 * form; the paper leaves the GPU kernel's shape open, section "Large Sparse Neural
 * Network Inference").  Times layer 0 over `rows` rows with every kernel variant of
 * the net's family that fits (variants of one family sum each output in the same
 * order, so the choice never changes results) and keeps the fastest; its time per
 * layer is reported as sdnn_plan.tuned_us.
 *   y_sample  dev fp32 [rows][N]: rows of the workload (e.g. the first batch), rows <=
 *             max_rows; or NULL: all-ones rows, min(rows, max_rows / 2) of them
 * Uses the workspace as scratch (a later forward rewrites it).  Synchronizes.
 * SDNN_EINVAL for rows < 0 or rows > max_rows with a sample. */
sdnn_status sdnn_tune(sdnn_net net, const float *y_sample, int64_t rows, void *stream);

/*
 * Forward pass over `rows` input rows.
 * Paper: section "Large Sparse Neural Network Inference" (the layered inference,
 * its batches of inputs dispatched by a loop of condition tasks, section
 * "Conditional Tasking", and the truth-category check of the result).
 *   y0        dev fp32 [rows][N]   input activations (not modified)
 *   batch_off host int64 [n_batches+1] ascending offsets, 0 .. rows, or NULL
 *             (one batch).  Batches are consecutive row ranges; rows are
 *             independent, so results never depend on the split.  With
 *             SDNN_EXEC_GRAPH / EAGER batches run one after another ("plain");
 *             with SDNN_EXEC_PERSISTENT all batches run in one launch.
 *   y_out     dev fp32 [rows][N]   final activations; rows that became all-zero
 *             are exactly zero.  Must not overlap y0.  Also used as one of the
 *             two ping-pong activation buffers.
 *   nz_rows   dev int32 [rows]     ascending ids of rows with a nonzero final
 *             activation (the "categories" output); entries past n_nz undefined.
 *   n_nz      dev int32 [1]        number of such rows.
 *   ckpt      dev fp32, sdnn_ckpt_size bytes, or NULL: receives Y_S, Y_2S, ...
 *             (rows alive at that layer) for sdnn_backward.
 *   layer_rows dev int32 [L+1] or NULL: layer_rows[l] = rows processed by layer l
 *             (layer 0 processes every row), layer_rows[L] = n_nz.
 */
sdnn_status sdnn_forward(sdnn_net net, const float *y0, int64_t rows, const int64_t *batch_off, int32_t n_batches,
                         float *y_out, int32_t *nz_rows, int32_t *n_nz, float *ckpt, int32_t *layer_rows,
                         void *stream);

/*
 * One layer over all `rows` rows, no compaction: y_out = min(c, max(0, y_in W_l + b_l)).
 * Used to check the forward layer by layer.  y_in/y_out dev fp32 [rows][N], must not overlap;
 * rows <= max_rows (the wide-layer kernels pack the rows into the workspace).
 * Paper: section "Large Sparse Neural Network Inference" (one layer of the rule).
 */
sdnn_status sdnn_layer(sdnn_net net, int32_t layer, const float *y_in, int64_t rows, float *y_out, void *stream);

/*
 * Backward pass of the last sdnn_forward over the same y0 / rows / ckpt (needs
 * SDNN_TRAINABLE).  Only rows listed in nz_rows can carry a gradient (every other
 * row is all-zero after some layer, where the mask 0 < y < c stops it), so the
 * pass runs on those rows, recomputing each checkpoint segment of S layers.
 *   nz_rows, n_nz  dev, as written by that forward
 *   dy_out    dev fp32 [rows][N]   dL/dY_L
 *   dw        dev fp32 [L][N][k]   dL/dw  (overwritten)
 *   dbias     dev fp32 [L][N]      dL/db  (overwritten)
 *   dy0       dev fp32 [rows][N] or NULL: dL/dY_0 (overwritten)
 * Deterministic: no floating-point atomics; every sum has a fixed order.
 * Paper: none (training is an extension of the layer rule of section "Large
 * Sparse Neural Network Inference").
 */
sdnn_status sdnn_backward(sdnn_net net, const float *y0, int64_t rows, const float *ckpt, const int32_t *nz_rows,
                          const int32_t *n_nz, const float *dy_out, float *dw, float *dbias, float *dy0,
                          void *stream);

/*
 * Backward pass of one layer over `rows` rows (needs SDNN_TRAINABLE), the same
 * kernels sdnn_backward chains:
 *   G = dy_out * [0 < y_out < c];  dbias[j] = sum_r G[r][j];
 *   dw[j][s] = sum_r G[r][j] y_in[r][idx[j][s]];  dy_in[r][i] = sum_{(j,s): idx[j][s]=i} G[r][j] w[j][s].
 *   y_in, y_out, dy_out dev fp32 [rows][N] (y_out = this layer's forward output);
 *   dw dev fp32 [N][k], dbias dev fp32 [N] (this layer's slices; overwritten);
 *   dy_in dev fp32 [rows][N] or NULL.  rows <= max_rows.
 * Paper: none (as sdnn_backward).
 */
sdnn_status sdnn_layer_backward(sdnn_net net, int32_t layer, const float *y_in, const float *y_out,
                                const float *dy_out, int64_t rows, float *dw, float *dbias, float *dy_in,
                                void *stream);

/*
 * Mean-squared-error loss of y against t (n elements) and its gradient:
 *   dy (dev fp32 [n], may be NULL) = 2 (y - t) / n
 *   loss (dev fp32 [257], may be NULL): loss[0] = sum (y - t)^2 / n; loss[1..256]
 *   are scratch for per-block partial sums.  The loss is reduced in a fixed order.
 * Paper: none (the training loss of the backward extension).
 */
sdnn_status sdnn_mse(const float *y, const float *t, int64_t n, float *dy, float *loss, void *stream);

/*
 * sdnn_mse for callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same result,
 * bitwise, with no scratch tail on `loss` and no allocation of any kind.
 *   y, t     dev fp32 [n]
 *   dy       dev fp32 [n] or NULL: 2 (y - t) / n
 *   loss     dev fp32 [1] or NULL: sum (y - t)^2 / n
 * The 256 per-workgroup partial sums live in a static device array of 1 KiB per
 * GPU (held until the process ends); that holds them for every n >= 0, so no size
 * is too large (n < 0 is SDNN_EINVAL).  Every call on one GPU shares that array:
 * calls that overlap on one GPU (other streams, other threads) race and must be
 * serialized by the caller.  The first call on a device looks up the array's
 * device address (SDNN_EHIP if that fails; device ordinals >= 64 are
 * SDNN_EUNSUPPORTED).
 */
sdnn_status sdnn_mse_noalloc(const float *y, const float *t, int64_t n, float *dy, float *loss, void *stream);

/*
 * Host-side slot schedule of the resident-weight forward kernel, as sdnn_create
 * builds it (no GPU involved).  For each block of 64 neurons the neurons are
 * spread over the four 16-lane LDS service units of a wave and each lane's 32
 * slots are ordered so that, at every step, the 16 lanes of a unit read 16
 * distinct LDS bank groups (input id mod 16); lanes are padded to the block's
 * step count with weight-0 steps.
 *   idx          host int32 [L][N][k] (ids in [0, N))
 *   ent          host uint32 [L][npad][dmax]: (id << 5) | slot, or a pad step
 *                (bit 31 set, id = a free bank group); npad = 64 * ceil(N / 64)
 *   lane_neuron  host int32 [L][npad]: neuron computed by each lane slot, -1 if none
 *   steps        host int32 [L][ceil(N / 64)]: steps of each block
 * Returns the largest block step count (> dmax: the schedule does not fit and the
 * entries past dmax were dropped), or SDNN_EINVAL / SDNN_EUNSUPPORTED.
 * Paper: none (a kernel-design detail of this library).
 */
int32_t sdnn_schedule_host(const int32_t *idx, int32_t n_neurons, int32_t n_layers, int32_t dmax, uint32_t *ent,
                           int32_t *lane_neuron, int32_t *steps);

/*
 * Host-side slot orders of the bank-scheduled one-row-tile kernel (plan variant 5),
 * as sdnn_create builds them (no GPU involved).  The kernel reads an activation row
 * from LDS with 4-byte reads, one slot per lane per step; a half-wave of 32 lanes
 * (32 consecutive neurons) is served in one pass when its lanes hit 32 distinct
 * banks (input id mod 32).  For every such block the orders take K "double" steps
 * (each bank at most two lanes) and 32 - K conflict-free steps, with K = max(max_b
 * d_b - 32, 32 - min_b d_b) for the block's per-bank slot counts d_b (a greedy
 * order for a partial last block).
 *   idx   host int32 [L][N][k], ids in [0, N)
 *   perm  host uint8 [L][N][k]: perm[l][j][step] = the slot neuron j reads at step
 * Returns the summed cost in LDS passes over all blocks (sum over steps of the
 * busiest bank's lane count), or SDNN_EINVAL (< 0) for bad arguments.
 * Paper: none (a kernel-design detail of this library).
 */
int64_t sdnn_row_schedule_host(const int32_t *idx, int32_t n_neurons, int32_t n_layers, uint8_t *perm);

/* Synchronize `stream` and report whether a kernel of this net raised its error word.
 * The word stays set: after SDNN_EDEVICE the net's scratch state (work lists, per-tile
 * counters of a layer that stopped part-way) is undefined, so destroy and recreate it.
 * Without a synchronization, the finalize pass of every sdnn_forward copies a raised
 * error word into pinned host memory, and sdnn_forward, sdnn_layer, sdnn_backward,
 * sdnn_layer_backward and sdnn_tune return SDNN_EDEVICE (launching nothing) once that
 * copy has landed, i.e. on the first call that starts after the failing forward has
 * finished on the device.  Paper: none (failure detection of this library). */
sdnn_status sdnn_check_device(sdnn_net net, void *stream);

/* Failure injection for tests of the error path: enqueue on `stream` a write of `code`
 * (nonzero) into the net's device error word, as a timed-out barrier would.  Every
 * persistent-kernel grid barrier then gives up at once (its kernel returns normally),
 * the next forward's finalize pass publishes the word, and the net must be recreated.
 * SDNN_EINVAL for a NULL net or code 0.  Paper: none (test support). */
sdnn_status sdnn_inject_device_error(sdnn_net net, int32_t code, void *stream);

/* Release the net (NULL-safe).  Does not free caller buffers.  Paper: none. */
void sdnn_destroy(sdnn_net net);

/* Thread-local message of the last failure.  Paper: none. */
const char *sdnn_last_error(void);

/* Library version string.  Paper: none. */
const char *sdnn_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SDNN_H */
