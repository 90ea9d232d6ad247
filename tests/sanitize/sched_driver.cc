// Sanitizer driver of the host-side schedule builders (built host-only): the
// bank-conflict slot schedules of the scheduled kernels (forward and transposed)
// and the slot order of the one-row-tile kernel, on random nets of several widths,
// including ragged ones (N not a multiple of 64).  Checks the structural facts each
// builder promises and prints "all ok".
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

namespace sdnn {
int build_schedule(const int32_t* idx, int N, int L, int dmax, uint32_t* ent, int32_t* lane_neuron,
                   int32_t* wave_steps);
int build_transposed_schedule(const int32_t* idx, int N, int L, int dmax, uint32_t* ent, int32_t* lane_input,
                              int32_t* wave_steps);
int64_t build_row_schedule(const int32_t* idx, int N, int L, uint8_t* perm);
}  // namespace sdnn

int main() {
    const int K = 32, DSTORE = 64;
    std::mt19937 rng(5);
    int bad = 0;
    for (int N : {64, 100, 1024, 2052}) {
        const int L = 3;
        std::vector<int32_t> idx((size_t)L * N * K);
        std::vector<int32_t> all(N);
        for (int i = 0; i < N; ++i) all[i] = i;
        for (int l = 0; l < L; ++l)
            for (int j = 0; j < N; ++j) {
                std::shuffle(all.begin(), all.end(), rng);
                std::sort(all.begin(), all.begin() + K);
                std::copy(all.begin(), all.begin() + K, idx.begin() + ((size_t)l * N + j) * K);
            }
        const int nblk = (N + 63) / 64;
        const size_t npad = (size_t)nblk * 64;
        std::vector<uint32_t> ent((size_t)L * npad * DSTORE);
        std::vector<int32_t> ln((size_t)L * npad), ws((size_t)L * nblk);
        const int worst = sdnn::build_schedule(idx.data(), N, L, DSTORE, ent.data(), ln.data(), ws.data());
        // every neuron appears on exactly one lane of each layer
        for (int l = 0; l < L; ++l) {
            std::vector<int> seen(N, 0);
            for (size_t s = 0; s < npad; ++s) {
                const int j = ln[(size_t)l * npad + s];
                if (j >= 0 && j < N) ++seen[j];
            }
            for (int j = 0; j < N; ++j) bad += seen[j] != 1;
        }
        std::vector<uint32_t> tent(ent.size());
        std::vector<int32_t> tln(ln.size()), tws(ws.size());
        const int tworst =
            sdnn::build_transposed_schedule(idx.data(), N, L, DSTORE, tent.data(), tln.data(), tws.data());
        std::vector<uint8_t> perm(idx.size());
        const long long cost = sdnn::build_row_schedule(idx.data(), N, L, perm.data());
        // each neuron's row-kernel order is a permutation of its 32 slots
        for (size_t j = 0; j < (size_t)L * N; ++j) {
            uint32_t m = 0;
            for (int s = 0; s < K; ++s) m |= 1u << perm[j * K + s];
            bad += m != 0xffffffffu;
        }
        printf("N=%d schedule worst %d transposed worst %d row cost %lld\n", N, worst, tworst, cost);
        bad += worst < K || tworst < 1 || cost < (long long)L * ((N + 31) / 32) * K;
    }
    printf(bad ? "FAILED %d\n" : "all ok\n", bad);
    return bad != 0;
}
