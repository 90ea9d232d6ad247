/*
 * FP64 reference implementation ("oracle") of the layered sparse DNN.
 *
 * TEST INFRASTRUCTURE ONLY: the GPU library never links, loads or calls this
 * file.  It shares no code, header or table with the GPU path.
 *
 * The paper (section "Large Sparse Neural Network Inference") runs inference of
 * the sparse-DNN challenge it cites: an input matrix pushed through a stack of
 * sparse layers with per-neuron bias values, checked against truth categories.
 * The paper does not write the layer rule out.  The rule taken here (the
 * challenge's rule, with K = 32 inputs per neuron and a clip at c = 32) is:
 * multiply the activations by the sparse layer matrix, add the bias, apply
 * ReLU, clip at c.  With W_l stored by output neuron (slot k of neuron j reads
 * input neuron idx[j][k] with weight w[j][k]):
 *
 *     z[r][j]          = sum_{k=0..K-1} w[j][k] * y_l[r][idx[j][k]]  +  b[j]
 *     y_{l+1}[r][j]    = min(c, max(0, z[r][j]))                     (c = 32)
 *
 * Parameters are taken as their exact fp32 values promoted to double; sums run
 * over slots in ascending order, bias last, in round-to-nearest double.
 *
 * The backward pass is the chain rule through the same rule, with the
 * derivative of min(c, max(0, z)) taken as 1 when 0 < z < c and 0 otherwise
 * (a function of the output alone: 0 < y < c):
 *
 *     G[r][j]          = dY_{l+1}[r][j] * [0 < y_{l+1}[r][j] < c]
 *     db[j]            = sum_r G[r][j]
 *     dW[j][k]         = sum_r G[r][j] * y_l[r][idx[j][k]]
 *     dY_l[r][i]       = sum_{(j,k) : idx[j][k] = i} G[r][j] * w[j][k]
 *
 * Forward error bound.  Any fp32 evaluation of one layer (products and sums in
 * any order, with or without fused multiply-adds) from inputs that differ from
 * the exact ones by at most e_in satisfies, to first order,
 *     |y_fp32 - y| <= (1 + g) sum_k |w| e_in[idx] + g (sum_k |w y| + |b|),
 * g = gamma_33 = 33u / (1 - 33u) (32 products and one bias add, u = 2^-24):
 * the sum of 33 rounded terms has error at most gamma_33 times the sum of their
 * magnitudes, the input errors pass through with the weights' magnitudes, and
 * min(c, max(0, .)) is 1-Lipschitz so it never enlarges an error.  Applying this
 * layer by layer gives a bound for the whole chain.
 *
 * Rows are independent: every function below treats the R rows it is given
 * and knows nothing of compaction, batches or checkpoints; the Python driver
 * next to this file strings layers together.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * One forward layer over R independent rows.
 *   y_in  [R][N] double     activations entering the layer
 *   y_out [R][N] double     activations leaving it
 *   z_out [R][N] double     pre-activation z (optional, NULL to skip)
 *   s_out [R][N] double     conditioning scale sum_k |w y| + |b| (optional)
 *   alive [R]   uint8       1 if the output row has a nonzero (optional)
 */
void orc_layer_forward(int64_t R, int32_t N, int32_t K,
                       const int32_t *idx, const float *w, const float *b, double clamp,
                       const double *y_in, double *y_out, double *z_out, double *s_out,
                       uint8_t *alive, int nthreads)
{
    set_threads(nthreads);
    int64_t r;
#pragma omp parallel for schedule(static)
    for (r = 0; r < R; ++r) {
        const double *yi = y_in + r * (int64_t)N;
        double *yo = y_out + r * (int64_t)N;
        int any = 0;
        for (int32_t j = 0; j < N; ++j) {
            const int32_t *ij = idx + (int64_t)j * K;
            const float *wj = w + (int64_t)j * K;
            double z = 0.0, s = 0.0;
            for (int32_t k = 0; k < K; ++k) {
                double t = (double)wj[k] * yi[ij[k]];
                z += t;
                s += fabs(t);
            }
            z += (double)b[j];
            s += fabs((double)b[j]);
            double y = z > 0.0 ? z : 0.0;
            if (y > clamp) y = clamp;
            yo[j] = y;
            if (z_out) z_out[r * (int64_t)N + j] = z;
            if (s_out) s_out[r * (int64_t)N + j] = s;
            if (y != 0.0) any = 1;
        }
        if (alive) alive[r] = (uint8_t)any;
    }
}

/*
 * One backward layer over R rows.
 *   y_in   [R][N]  activations entering the layer (forward values)
 *   y_out  [R][N]  activations leaving it (defines the mask 0 < y < c)
 *   dy_out [R][N]  gradient of the loss w.r.t. y_out
 *   dw     [N][K]  gradient w.r.t. w (overwritten)
 *   db     [N]     gradient w.r.t. b (overwritten)
 *   dy_in  [R][N]  gradient w.r.t. y_in (overwritten; optional)
 */
void orc_layer_backward(int64_t R, int32_t N, int32_t K,
                        const int32_t *idx, const float *w, double clamp,
                        const double *y_in, const double *y_out, const double *dy_out,
                        double *dw, double *db, double *dy_in, int nthreads)
{
    set_threads(nthreads);
    int32_t j;
    /* db and dW: one neuron per iteration, rows summed in ascending order. */
#pragma omp parallel for schedule(static)
    for (j = 0; j < N; ++j) {
        const int32_t *ij = idx + (int64_t)j * K;
        double sb = 0.0;
        double *dwj = dw + (int64_t)j * K;
        for (int32_t k = 0; k < K; ++k) dwj[k] = 0.0;
        for (int64_t r = 0; r < R; ++r) {
            double y = y_out[r * (int64_t)N + j];
            double g = (y > 0.0 && y < clamp) ? dy_out[r * (int64_t)N + j] : 0.0;
            if (g == 0.0) continue;
            sb += g;
            const double *yi = y_in + r * (int64_t)N;
            for (int32_t k = 0; k < K; ++k) dwj[k] += g * yi[ij[k]];
        }
        db[j] = sb;
    }
    if (!dy_in) return;
    /* dY_in: scatter each row's masked gradient through the transposed pattern. */
    int64_t r;
#pragma omp parallel for schedule(static)
    for (r = 0; r < R; ++r) {
        double *di = dy_in + r * (int64_t)N;
        const double *yo = y_out + r * (int64_t)N;
        const double *go = dy_out + r * (int64_t)N;
        for (int32_t i = 0; i < N; ++i) di[i] = 0.0;
        for (int32_t jj = 0; jj < N; ++jj) {
            double y = yo[jj];
            if (!(y > 0.0 && y < clamp)) continue;
            double g = go[jj];
            const int32_t *ij = idx + (int64_t)jj * K;
            const float *wj = w + (int64_t)jj * K;
            for (int32_t k = 0; k < K; ++k) di[ij[k]] += g * (double)wj[k];
        }
    }
}

/*
 * Propagate the forward error bound through one layer (see the header):
 *   e_out[r][j] = (1 + g) sum_k |w[j][k]| e_in[r][idx[j][k]] + g (sum_k |w[j][k] y_in[r][idx[j][k]]| + |b[j]|)
 * y_in are the exact (double) activations entering the layer; e_in may be NULL (exact inputs).
 */
void orc_layer_bound(int64_t R, int32_t N, int32_t K, const int32_t *idx, const float *w, const float *b, double g,
                     const double *y_in, const double *e_in, double *e_out, int nthreads)
{
    set_threads(nthreads);
    int64_t r;
#pragma omp parallel for schedule(static)
    for (r = 0; r < R; ++r) {
        const double *yi = y_in + r * (int64_t)N;
        const double *ei = e_in ? e_in + r * (int64_t)N : NULL;
        double *eo = e_out + r * (int64_t)N;
        for (int32_t j = 0; j < N; ++j) {
            const int32_t *ij = idx + (int64_t)j * K;
            const float *wj = w + (int64_t)j * K;
            double prop = 0.0, s = 0.0;
            for (int32_t k = 0; k < K; ++k) {
                double aw = fabs((double)wj[k]);
                s += aw * fabs(yi[ij[k]]);
                if (ei) prop += aw * ei[ij[k]];
            }
            s += fabs((double)b[j]);
            eo[j] = (1.0 + g) * prop + g * s;
        }
    }
}
