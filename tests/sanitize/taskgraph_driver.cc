// Sanitizer driver of the task-graph executor on the CPU (built against the
// stand-in HIP header): diamond chains over CPU and GPU-domain workers, loops of
// condition tasks, and the inference pipeline with a stand-in forward (its nonzero
// rows are the rows with at least 3 ones), over repeated executor lifetimes.
// Prints "all ok" and exits 0 when every result is right.
#include <cstdio>
#include <cstdint>
#include <vector>
#include <cstring>
#include "sdnn_taskgraph.h"

struct sdnn_net_s { int N; };
static thread_local char err[64] = "none";
extern "C" const char* sdnn_last_error(void) { return err; }
// stand-in forward: y = y0; nonzero rows = rows with at least 3 ones
extern "C" sdnn_status sdnn_forward(sdnn_net net, const float* y0, int64_t rows, const int64_t*, int32_t,
                                    float* y, int32_t* nz, int32_t* n_nz, float*, int32_t*, void*) {
    const int N = net->N;
    int32_t c = 0;
    for (int64_t r = 0; r < rows; ++r) {
        int ones = 0;
        for (int j = 0; j < N; ++j) { y[r * N + j] = y0[r * N + j]; ones += y0[r * N + j] != 0; }
        if (ones >= 3) nz[c++] = (int32_t)r;
    }
    *n_nz = c;
    return SDNN_OK;
}

static int64_t expected_sum(int w, int d) {
    int64_t s = 2;
    for (int l = 0; l < d; ++l) for (int i = 0; i < w; ++i) s += (int64_t)l * w + i + 2;
    return s;
}

int main() {
    int bad = 0;
    for (int rep = 0; rep < 6; ++rep) {
        sdnn_tg_executor ex;
        if (sdnn_tg_executor_create(1 + rep % 4, rep % 3, &ex)) { printf("create: %s\n", sdnn_tg_last_error()); return 1; }
        for (int k = 0; k < 20; ++k) {
            int64_t s = 0;
            const int w = 1 + (k * 7) % 13, d = 1 + (k * 5) % 9;
            const int ge = (rep % 3) ? (k % 4) : 0;
            if (sdnn_tg_run_diamond_chain(ex, w, d, ge, &s) || s != expected_sum(w, d)) { ++bad; printf("diamond %d %d\n", w, d); }
            int32_t c = -1;
            if (sdnn_tg_run_condition_loop(ex, k, &c) || c != (k ? k : 1)) { ++bad; printf("loop %d -> %d\n", k, c); }
        }
        if (rep % 3) {
            const int N = 24, R = 300, nb = 7, ngpu = rep % 3;
            std::vector<int64_t> off{0, 10, 10, 90, 91, 200, 260, 300};
            std::vector<int64_t> ptr(R + 1, 0);
            std::vector<int32_t> cols;
            std::vector<int64_t> toff(nb + 1, 0);
            std::vector<int32_t> trows;
            for (int r = 0; r < R; ++r) {
                const int n = (r * 37) % 6;
                for (int e = 0; e < n; ++e) cols.push_back((r * 11 + e * 5) % N);
                ptr[r + 1] = (int64_t)cols.size();
            }
            for (int b = 0; b < nb; ++b) {
                for (int64_t r = off[b]; r < off[b + 1]; ++r) if ((r * 37) % 6 >= 3) trows.push_back((int32_t)r);
                toff[b + 1] = (int64_t)trows.size();
            }
            std::vector<sdnn_net_s> nets(ngpu, sdnn_net_s{N});
            std::vector<sdnn_net> hs;
            for (auto& n : nets) hs.push_back(&n);
            std::vector<float> y0((size_t)R * N), y((size_t)R * N);
            std::vector<int32_t> nz(R), nnz(nb);
            std::vector<int64_t> mism(nb);
            for (int k = 0; k < 5; ++k) {
                double sec = 0;
                if (sdnn_tg_pipeline_run(ex, hs.data(), ngpu, N, R, off.data(), nb, ptr.data(), cols.data(), toff.data(),
                                         trows.empty() ? nullptr : trows.data(), y0.data(), y.data(), nz.data(), nnz.data(),
                                         mism.data(), &sec)) { printf("pipeline: %s\n", sdnn_tg_last_error()); return 1; }
                for (int b = 0; b < nb; ++b) if (mism[b]) { ++bad; printf("mism batch %d: %lld\n", b, (long long)mism[b]); }
            }
        }
        int64_t st[4];
        sdnn_tg_executor_stats(ex, st);
        printf("rep %d: executed %lld steals %lld failed %lld sleeps %lld\n", rep, (long long)st[0], (long long)st[1],
               (long long)st[2], (long long)st[3]);
        sdnn_tg_executor_destroy(ex);
    }
    printf(bad ? "FAILED %d\n" : "all ok\n", bad);
    return bad != 0;
}
