// Sanitizer driver of the host-side schedule builders (built host-only): the
// bank-conflict slot schedules of the scheduled kernels (forward and transposed),
// the slot order of the one-row-tile kernel, and the neuron pairs of the chunked
// one-row-tile kernel, on random nets of several widths, including ragged ones (N
// not a multiple of 64).  Checks the structural facts each builder promises and
// prints "all ok".
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
int build_rowc_pairs(const uint32_t* counts, int N, int L, int C, uint32_t* pairs);
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
    // neuron pairs of the chunked kernel: every neuron of a part in exactly one pair,
    // pairs in order of non-increasing overflow, the returned overflow is the largest
    // part's, and it fits the LDS list
    for (int N : {20480, 32768, 65536}) {
        const int L = 2, C = N <= 32768 ? 2 : 4, CW = N / C, PC = 64 / C, PART = 2048;
        std::vector<uint32_t> cnt((size_t)L * N);
        std::vector<int32_t> all(N);
        for (int i = 0; i < N; ++i) all[i] = i;
        for (size_t j = 0; j < cnt.size(); ++j) {
            for (int k = 0; k < K; ++k) std::swap(all[k], all[k + rng() % (N - k)]);
            uint32_t c = 0;
            for (int k = 0; k < K; ++k) c += 1u << (8 * (all[k] / CW));
            cnt[j] = c;
        }
        std::vector<uint32_t> pairs((size_t)L * N / 2);
        const int worst = sdnn::build_rowc_pairs(cnt.data(), N, L, C, pairs.data());
        int mine = 0;
        for (int l = 0; l < L; ++l)
            for (int p = 0; p < N / PART; ++p) {
                std::vector<int> seen(PART, 0);
                int ov = 0, prev = 1 << 30;
                for (int i = 0; i < PART / 2; ++i) {
                    const uint32_t pr = pairs[(size_t)l * N / 2 + (size_t)p * PART / 2 + i];
                    const int a = (int)(pr & 0xffffu), b = (int)(pr >> 16);
                    bad += a >= PART || b >= PART;
                    if (a >= PART || b >= PART) continue;
                    ++seen[a];
                    ++seen[b];
                    const uint32_t ca = cnt[(size_t)l * N + p * PART + a], cb = cnt[(size_t)l * N + p * PART + b];
                    int mine_ov = 0;
                    for (int c = 0; c < C; ++c) {
                        const int t = (int)((ca >> (8 * c)) & 255u) + (int)((cb >> (8 * c)) & 255u);
                        mine_ov += t > PC ? t - PC : 0;
                    }
                    bad += mine_ov > prev;
                    prev = mine_ov;
                    ov += mine_ov;
                }
                for (int j = 0; j < PART; ++j) bad += seen[j] != 1;
                mine = std::max(mine, ov);
            }
        printf("N=%d chunks %d: largest overflow list %d entries\n", N, C, worst);
        bad += worst != mine || worst > 2016;
    }
    printf(bad ? "FAILED %d\n" : "all ok\n", bad);
    return bad != 0;
}
