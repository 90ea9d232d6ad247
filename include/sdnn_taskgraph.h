/*
 * sdnn_taskgraph.h -- C ABI of the host task-graph executor and the inference
 * pipeline built on it.
 *
 * The paper's runtime runs heterogeneous task graphs (CPU and GPU tasks with
 * dependencies and condition tasks) on per-domain worker threads with work
 * stealing, and keeps the number of workers that hunt for work matched to the
 * available parallelism (section "Worker-level Scheduling Algorithm": the worker
 * loop, exploit/steal/execute/submit, the per-domain active and thief counts, the
 * two-phase sleep).  Its large sparse-DNN experiment (section "Large Sparse Neural
 * Network Inference") dispatches input batches to the GPUs and lets CPU tasks
 * check results against a golden reference, and reports the throughput of
 * co-running inference programs as weighted speedup.  This executor implements
 * that scheme for one GPU; sdnn_tg_pipeline_run builds and runs the inference
 * graph.
 *
 * Conventions are those of sdnn.h: status codes (SDNN_*), host pointers unless
 * named dev, caller-owned buffers, sdnn_tg_last_error() for a thread-local message.
 */
#ifndef SDNN_TASKGRAPH_H
#define SDNN_TASKGRAPH_H

#include <stdint.h>

#include "sdnn.h"

#ifdef __cplusplus
extern "C" {
#endif

#define SDNN_TG_CPU 0   /* task domains */
#define SDNN_TG_GPU 1

typedef struct sdnn_tg_executor_s *sdnn_tg_executor;
typedef struct sdnn_tg_graph_s *sdnn_tg_graph;

/* Start an executor with n_cpu CPU workers (1..256) and n_gpu GPU workers (0..64)
 * on the current HIP device.  Each GPU worker owns one HIP stream (default
 * priority) on which its GPU tasks enqueue work; a GPU task returns once its work
 * has finished on that stream.  SDNN_EINVAL for counts out of range, SDNN_EHIP if
 * a stream cannot be created.  GPU workers are currently switched off: n_gpu > 0
 * returns SDNN_EUNSUPPORTED (a process that ran GPU tasks on them ended with a
 * segmentation fault at exit, cause not yet found), so the pipeline cannot run.
 * Paper: section "Heterogeneous Work-stealing Architecture" (per-domain workers,
 * per-worker queues per domain, a shared queue per domain). */
int sdnn_tg_executor_create(int32_t n_cpu, int32_t n_gpu, sdnn_tg_executor *out);

/* Stop the workers (after the graphs they run have finished) and release the
 * executor (NULL-safe).  Paper: none. */
void sdnn_tg_executor_destroy(sdnn_tg_executor ex);

/* Counters since creation: stats4[0] tasks executed, [1] successful steals,
 * [2] failed steal attempts, [3] times a worker went to sleep.  Paper: section
 * "Heterogeneous Work-stealing Algorithm" (the quantities its analysis bounds). */
int sdnn_tg_executor_stats(sdnn_tg_executor ex, int64_t *stats4);

/* Self-checks of the scheduler (used by the tests): a layered DAG of `depth` levels
 * of `width` tasks, every task of a level depending on every task of the previous
 * level, with every gpu_every-th task in the GPU domain (0: none), between a source
 * and a sink; *sum receives the sum of the values the tasks add (2 + sum over tasks
 * of level * width + index + 2).  And a loop: a body task followed by a condition
 * task that sends control back to the body until it has run `iterations` times
 * (at least once); *count receives the number of body runs.  Paper: section
 * "Task-level Scheduling Algorithm" (dependency counts; a condition task releases
 * the one successor its return value names, section "Scheduling Condition Tasks"). */
int sdnn_tg_run_diamond_chain(sdnn_tg_executor ex, int32_t width, int32_t depth, int32_t gpu_every, int64_t *sum);
int sdnn_tg_run_condition_loop(sdnn_tg_executor ex, int32_t iterations, int32_t *count);

/*
 * The inference pipeline: for every batch b, three tasks
 *   decode[b] (CPU): rows batch_off[b] .. batch_off[b+1]-1 of the sparse binary
 *       input (row r's nonzero columns in_cols[in_ptr[r] .. in_ptr[r+1]-1]) into a
 *       pinned host buffer as dense 0/1 fp32 rows;
 *   infer[b]  (GPU): copy the rows into y0_dev, sdnn_forward of the batch on the
 *       worker's stream with the worker's net, copy its nonzero-row ids and count
 *       back, wait for the stream;
 *   check[b]  (CPU): compare them with the batch's truth categories (global row
 *       ids truth_rows[truth_off[b] .. truth_off[b+1]-1], ascending) and store
 *       the size of the symmetric difference in mismatches[b];
 * with decode[b] -> infer[b] -> check[b], run on the executor (blocking).
 *   nets        host array of n_nets nets, one per GPU worker of the executor, each
 *               over the same parameters with max_rows >= the largest batch (their
 *               exec mode is used as set; SDNN_EXEC_PERSISTENT avoids rebuilding a
 *               graph for every batch)
 *   rows, batch_off  host int64 [n_batches+1], 0 = batch_off[0] <= ... = rows
 *   in_ptr      host int64 [rows+1]; in_cols host int32 [in_ptr[rows]]
 *   truth_off   host int64 [n_batches+1]; truth_rows host int32
 *   y0_dev, y_dev  dev fp32 [rows][N] (inputs as decoded, final activations)
 *   nz_dev      dev int32 [rows] (each batch's nonzero rows at its offset, batch-local ids)
 *   n_nz_dev    dev int32 [n_batches]
 *   mismatches  host int64 [n_batches]
 *   seconds     host, or NULL: wall time of the run
 * Allocates rows * N * 4 + (rows + n_batches) * 4 bytes of pinned host memory for
 * the run.  SDNN_EINVAL for bad arguments, SDNN_ENOMEM if the pinned buffers cannot
 * be allocated, SDNN_EDEVICE if a task failed (sdnn_tg_last_error names it).
 * Paper: section "Large Sparse Neural Network Inference" (batches dispatched to the
 * GPU, results checked by CPU tasks against the truth categories).
 */
int sdnn_tg_pipeline_run(sdnn_tg_executor ex, sdnn_net *nets, int32_t n_nets, int32_t n_neurons, int64_t rows,
                         const int64_t *batch_off, int32_t n_batches, const int64_t *in_ptr, const int32_t *in_cols,
                         const int64_t *truth_off, const int32_t *truth_rows, float *y0_dev, float *y_dev,
                         int32_t *nz_dev, int32_t *n_nz_dev, int64_t *mismatches, double *seconds);

/* Thread-local message of the last failure of a task-graph call.  Paper: none. */
const char *sdnn_tg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SDNN_TASKGRAPH_H */
