/* Sanitizer driver of the oracle's C core (built with the address and undefined
 * behaviour sanitizers): forward, backward and bound propagation over small random
 * nets with ragged widths, each run on 1 and 4 threads, checking that both runs
 * agree exactly and that a one-layer forward matches a dense recomputation.
 * Prints "all ok". */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void orc_layer_forward(int64_t R, int32_t N, int32_t K, const int32_t *idx, const float *w, const float *b,
                       double clamp, const double *y_in, double *y_out, double *z_out, double *s_out, uint8_t *alive,
                       int nthreads);
void orc_layer_backward(int64_t R, int32_t N, int32_t K, const int32_t *idx, const float *w, double clamp,
                        const double *y_in, const double *y_out, const double *dy_out, double *dw, double *db,
                        double *dy_in, int nthreads);
void orc_layer_bound(int64_t R, int32_t N, int32_t K, const int32_t *idx, const float *w, const float *b, double g,
                     const double *y_in, const double *e_in, double *e_out, int nthreads);

static uint64_t st = 88172645463325252ull;
static uint64_t rnd(void) { st ^= st << 13; st ^= st >> 7; st ^= st << 17; return st; }
static double unif(void) { return (double)(rnd() >> 11) / 9007199254740992.0; }

int main(void) {
    int bad = 0;
    const int sizes[][3] = {{37, 40, 8}, {5, 64, 32}, {64, 33, 32}, {1, 70, 3}};
    for (int c = 0; c < 4; ++c) {
        const int R = sizes[c][0], N = sizes[c][1], K = sizes[c][2];
        int32_t *idx = malloc(sizeof(int32_t) * N * K);
        float *w = malloc(sizeof(float) * N * K), *b = malloc(sizeof(float) * N);
        double *y0 = malloc(sizeof(double) * R * N), *y1 = malloc(sizeof(double) * R * N);
        double *y1b = malloc(sizeof(double) * R * N), *z = malloc(sizeof(double) * R * N);
        double *s = malloc(sizeof(double) * R * N), *dy = malloc(sizeof(double) * R * N);
        double *dw = malloc(sizeof(double) * N * K), *dw4 = malloc(sizeof(double) * N * K);
        double *db = malloc(sizeof(double) * N), *db4 = malloc(sizeof(double) * N);
        double *dyi = malloc(sizeof(double) * R * N), *dyi4 = malloc(sizeof(double) * R * N);
        double *e = malloc(sizeof(double) * R * N), *e2 = malloc(sizeof(double) * R * N);
        uint8_t *alive = malloc((size_t)R);
        for (int j = 0; j < N; ++j) {
            /* K distinct ascending ids: a random subset by selection sampling */
            int k = 0;
            for (int i = 0; i < N && k < K; ++i)
                if (unif() * (N - i) < (K - k)) idx[j * K + k++] = i;
            for (int q = 0; q < K; ++q) w[j * K + q] = (float)(unif() * 0.2 - 0.05);
            b[j] = (float)(-0.1 * unif());
        }
        for (int i = 0; i < R * N; ++i) { y0[i] = unif() < 0.3 ? 1.0 : 0.0; dy[i] = unif() - 0.5; }
        orc_layer_forward(R, N, K, idx, w, b, 32.0, y0, y1, z, s, alive, 1);
        orc_layer_forward(R, N, K, idx, w, b, 32.0, y0, y1b, NULL, NULL, NULL, 4);
        bad += memcmp(y1, y1b, sizeof(double) * R * N) != 0;
        for (int r = 0; r < R; ++r)
            for (int j = 0; j < N; ++j) {
                double zz = 0.0;
                for (int i = 0; i < N; ++i) {
                    double wd = 0.0;
                    for (int q = 0; q < K; ++q) if (idx[j * K + q] == i) wd = w[j * K + q];
                    zz += wd * y0[r * N + i];
                }
                zz += b[j];
                const double y = zz < 0.0 ? 0.0 : (zz > 32.0 ? 32.0 : zz);
                bad += fabs(y - y1[r * N + j]) > 1e-12;
            }
        orc_layer_backward(R, N, K, idx, w, 32.0, y0, y1, dy, dw, db, dyi, 1);
        orc_layer_backward(R, N, K, idx, w, 32.0, y0, y1, dy, dw4, db4, dyi4, 4);
        bad += memcmp(dw, dw4, sizeof(double) * N * K) != 0 || memcmp(db, db4, sizeof(double) * N) != 0 ||
               memcmp(dyi, dyi4, sizeof(double) * R * N) != 0;
        orc_layer_bound(R, N, K, idx, w, b, 1e-7, y0, NULL, e, 1);
        orc_layer_bound(R, N, K, idx, w, b, 1e-7, y1, e, e2, 4);
        for (int i = 0; i < R * N; ++i) bad += !(e[i] >= 0.0) || !(e2[i] >= 0.0);
        printf("R=%d N=%d K=%d done\n", R, N, K);
        free(idx); free(w); free(b); free(y0); free(y1); free(y1b); free(z); free(s); free(dy); free(dw); free(dw4);
        free(db); free(db4); free(dyi); free(dyi4); free(e); free(e2); free(alive);
    }
    printf(bad ? "FAILED %d\n" : "all ok\n", bad);
    return bad != 0;
}
