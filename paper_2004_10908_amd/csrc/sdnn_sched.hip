// Create-time slot scheduling for the resident-weight forward kernel.
//
// The scheduled kernel stages 4 activation rows per tile in LDS, [id][row], so
// the 4 values one input id feeds are one 16-byte slot whose bank group is
// id mod 16.
// On gfx950 a 16-byte LDS read is served 16 lanes per cycle against 64 banks,
// in four fixed lane units made of lane quads: unit 2h + p holds the quads
// (lanes 4c .. 4c+3) of half-wave h whose index c = 0..7 within the half has bit
// parity p, e.g. unit 0 = {0-3, 12-15, 20-23, 24-27}.  A unit's read is
// conflict-free iff its 16 lanes hit 16 distinct bank groups (slot mod 16).
// (Measured on the device with the LDS bank-conflict counter: exchanging the bank
// groups of two lanes of a conflict-free pattern stays conflict-free exactly when
// both lanes are in the same unit.)
//
// Each lane owns one neuron for a whole layer and may process its 32 slots in
// any order.  For every block of 64 neurons (one wave) this file:
//   1. balances the 64 neurons over the 4 units so that each unit's per-group
//      slot counts are as even as possible (greedy + pairwise swaps): the number
//      of steps a unit needs is at least its largest group count;
//   2. schedules each unit greedily: at every step each lane takes a slot whose
//      group no other lane of the unit uses in that step (the lane with most
//      remaining slots picks first, its most frequent free group);
//   3. pads every lane to the block's step count with dummy steps (weight 0) that
//      read a group left free in that step, keeping every step conflict-free.
// The summation order of a neuron is therefore its schedule order, fixed at
// create time: results are deterministic and identical across engines.
#include <algorithm>
#include <array>
#include <atomic>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

#include "sdnn_internal.hpp"

namespace sdnn {

namespace {

constexpr int NG = 16;        // bank groups of 16 bytes
constexpr int UNITS = 4;      // lane units per wave
constexpr int ULANES = 16;    // lanes per unit

// wave lane of position q (0..15) in unit u
inline int unit_lane(int u, int q) {
    static const int quads[2][4] = {{0, 3, 5, 6}, {1, 2, 4, 7}};   // quads of a half-wave by bit parity
    return 32 * (u / 2) + 4 * quads[u % 2][q / 4] + (q % 4);
}

struct Block {
    int n = 0;                                  // real neurons in the block
    std::array<std::array<int, NG>, 64> hist{};  // per neuron, slots per group
};

// assign 64 neuron slots (some phantom) to 4 units of 16 -> unit_of[64]
void balance(const Block& B, std::array<int, 64>& members_out) {
    std::array<int, 64> order;
    for (int i = 0; i < 64; ++i) order[i] = i;
    auto mx = [&](int i) { return *std::max_element(B.hist[i].begin(), B.hist[i].end()); };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return mx(a) > mx(b); });
    std::array<std::array<int, NG>, UNITS> sum{};
    std::array<std::vector<int>, UNITS> mem;
    for (int i : order) {
        int best = -1, bv = 1 << 30;
        for (int u = 0; u < UNITS; ++u) {
            if ((int)mem[u].size() >= ULANES) continue;
            int v = 0;
            for (int g = 0; g < NG; ++g) v = std::max(v, sum[u][g] + B.hist[i][g]);
            if (v < bv) { bv = v; best = u; }
        }
        mem[best].push_back(i);
        for (int g = 0; g < NG; ++g) sum[best][g] += B.hist[i][g];
    }
    // Pairwise swaps between units: accept a swap that lowers the larger of the two
    // units' busiest-group counts, or keeps it and lowers their sum (plateau moves).
    auto umax = [&](int u) { return *std::max_element(sum[u].begin(), sum[u].end()); };
    for (int pass = 0; pass < 64; ++pass) {
        bool improved = false;
        for (int u1 = 0; u1 < UNITS; ++u1) {
            for (int u2 = u1 + 1; u2 < UNITS; ++u2) {
                int m1 = umax(u1), m2 = umax(u2);
                for (int a = 0; a < ULANES; ++a) {
                    for (int b = 0; b < ULANES; ++b) {
                        const int ia = mem[u1][a], ib = mem[u2][b];
                        int n1 = 0, n2 = 0;
                        for (int g = 0; g < NG; ++g) {
                            const int d = B.hist[ib][g] - B.hist[ia][g];
                            n1 = std::max(n1, sum[u1][g] + d);
                            n2 = std::max(n2, sum[u2][g] - d);
                        }
                        const int oldm = std::max(m1, m2), newm = std::max(n1, n2);
                        if (newm < oldm || (newm == oldm && n1 + n2 < m1 + m2)) {
                            for (int g = 0; g < NG; ++g) {
                                const int d = B.hist[ib][g] - B.hist[ia][g];
                                sum[u1][g] += d;
                                sum[u2][g] -= d;
                            }
                            std::swap(mem[u1][a], mem[u2][b]);
                            m1 = n1;
                            m2 = n2;
                            improved = true;
                        }
                    }
                }
            }
        }
        if (!improved) break;
    }
    for (int u = 0; u < UNITS; ++u)
        for (int q = 0; q < ULANES; ++q) members_out[unit_lane(u, q)] = mem[u][q];
}

}  // namespace

// One scheduled item: the bank group of the LDS slot a lane reads, and what the
// caller stores for it.
struct Item {
    int group;
    uint32_t payload;
};

// Schedule one block of up to 64 lanes; lists[i] are the items of block-local
// lane i (i < n).  Fills member[wave lane] (block-local index, >= n: none) and
// seq[wave lane] (payloads, or 0x80000000 | group for padding steps).
int schedule_block(const std::array<std::vector<Item>, 64>& lists, int n, std::array<int, 64>& member,
                   std::array<std::vector<uint32_t>, 64>& seq) {
    Block B;
    B.n = n;
    for (int i = 0; i < n; ++i)
        for (const Item& it : lists[i]) B.hist[i][it.group]++;
    balance(B, member);
    std::array<std::array<std::vector<uint32_t>, NG>, 64> pend;
    std::array<int, 64> left{};
    for (int lane = 0; lane < 64; ++lane) {
        seq[lane].clear();
        const int i = member[lane];
        if (i >= n) continue;
        for (const Item& it : lists[i]) {
            pend[lane][it.group].push_back(it.payload);
            ++left[lane];
        }
    }
    int steps_blk = 0;
    for (int u = 0; u < UNITS; ++u) {
        int lanes[ULANES];
        for (int q = 0; q < ULANES; ++q) lanes[q] = unit_lane(u, q);
        int remaining = 0;
        for (int q = 0; q < ULANES; ++q) remaining += left[lanes[q]];
        while (remaining > 0) {
            bool used[NG] = {};
            int pick[ULANES];
            int ord[ULANES];
            for (int q = 0; q < ULANES; ++q) ord[q] = q;
            std::stable_sort(ord, ord + ULANES, [&](int a, int c) { return left[lanes[a]] > left[lanes[c]]; });
            for (int oi = 0; oi < ULANES; ++oi) {
                const int q = ord[oi], lane = lanes[q];
                pick[q] = -1;
                int bg = -1, bc = 0;
                for (int g = 0; g < NG; ++g) {
                    const int c = (int)pend[lane][g].size();
                    if (c > bc && !used[g]) { bc = c; bg = g; }
                }
                if (bg >= 0) { used[bg] = true; pick[q] = bg; }
            }
            for (int q = 0; q < ULANES; ++q) {
                const int lane = lanes[q];
                if (pick[q] >= 0) {
                    seq[lane].push_back(pend[lane][pick[q]].back());
                    pend[lane][pick[q]].pop_back();
                    --left[lane];
                    --remaining;
                } else {
                    int g = 0;
                    while (used[g]) ++g;
                    used[g] = true;
                    seq[lane].push_back(0x80000000u | (uint32_t)g);
                }
            }
        }
        steps_blk = std::max(steps_blk, (int)seq[lanes[0]].size());
    }
    // pad to the block's step count: all 16 lanes of a unit take distinct groups
    for (int u = 0; u < UNITS; ++u)
        for (int q = 0; q < ULANES; ++q) {
            auto& sq = seq[unit_lane(u, q)];
            while ((int)sq.size() < steps_blk) sq.push_back(0x80000000u | (uint32_t)q);
        }
    return steps_blk;
}

// Forward schedule of layers [l0, l1).  idx: host copy of all ids [L][N][K].
//   ent[(l*npad + lane_slot)*dmax + s] = (id << 5) | k, or padding (bit 31 set, id = free group, k = 31)
//   lane_neuron[l*npad + lane_slot]   = neuron computed by that lane slot, or -1
//   wave_steps[l*nblk + b]            = steps of block b
// Returns the largest step count seen (callers reject > dmax).
int build_schedule_range(const int32_t* idx, int N, int l0, int l1, int dmax, uint32_t* ent, int32_t* lane_neuron,
                         int32_t* wave_steps) {
    const int nblk = (N + 63) / 64, npad = nblk * 64;
    int worst = 0;
    std::array<std::vector<Item>, 64> lists;
    std::array<int, 64> member;
    std::array<std::vector<uint32_t>, 64> seq;
    for (int l = l0; l < l1; ++l) {
        const int32_t* il = idx + (size_t)l * N * K;
        for (int b = 0; b < nblk; ++b) {
            const int n = std::min(64, N - 64 * b);
            for (int i = 0; i < 64; ++i) {
                lists[i].clear();
                if (i >= n) continue;
                for (int k = 0; k < K; ++k) {
                    const int32_t id = il[(size_t)(64 * b + i) * K + k];
                    lists[i].push_back({id % NG, ((uint32_t)id << 5) | (uint32_t)k});
                }
            }
            const int steps = schedule_block(lists, n, member, seq);
            worst = std::max(worst, steps);
            wave_steps[(size_t)l * nblk + b] = steps;
            for (int lane = 0; lane < 64; ++lane) {
                const size_t slot = (size_t)l * npad + 64 * b + lane;
                lane_neuron[slot] = member[lane] < n ? 64 * b + member[lane] : -1;
                for (int s = 0; s < dmax; ++s) {
                    uint32_t e = 0x80000000u | 31u;
                    if (s < (int)seq[lane].size()) {
                        e = seq[lane][s];
                        if (e & 0x80000000u) e = 0x80000000u | ((e & 0xffu) << 5) | 31u;
                    }
                    ent[slot * dmax + s] = e;
                }
            }
        }
    }
    return worst;
}

// Transposed schedule of layers [l0, l1) (for the input-gradient gather): lane
// slots are input neurons i, items are the edges (j, k) with idx[j][k] = i, read
// from the gradient tile at column j (bank group j mod 16).  Out-degrees vary
// (about 32 +- 6 for uniform patterns) and a block takes as many steps as its
// busiest lane, so the two blocks of a wave (neurons 128m .. 128m + 127) are
// formed by degree: the even block takes the 64 highest-degree neurons, the odd
// block the rest.  Both stay within the wave's 128 neurons, so the kernel's
// per-wave output staging is unchanged.
//   ent[...] = edge position j*K + k, or padding (bit 31 set, j*K = free group * K)
int build_transposed_range(const int32_t* idx, int N, int l0, int l1, int dmax, uint32_t* ent, int32_t* lane_input,
                           int32_t* wave_steps) {
    const int nblk = (N + 63) / 64, npad = nblk * 64;
    int worst = 0;
    std::vector<std::vector<uint32_t>> in_edges(N);
    std::array<std::vector<Item>, 64> lists;
    std::array<int, 64> member;
    std::array<std::vector<uint32_t>, 64> seq;
    std::vector<int> order;
    for (int l = l0; l < l1; ++l) {
        const int32_t* il = idx + (size_t)l * N * K;
        for (auto& v : in_edges) v.clear();
        for (int j = 0; j < N; ++j)
            for (int k = 0; k < K; ++k) in_edges[il[(size_t)j * K + k]].push_back((uint32_t)(j * K + k));
        for (int b = 0; b < nblk; ++b) {
            if ((b & 1) == 0) {
                // neurons of the block pair, by degree (descending; ties by id)
                const int lo = 64 * b, hi = std::min(N, 64 * b + 128);
                order.clear();
                for (int i = lo; i < hi; ++i) order.push_back(i);
                std::stable_sort(order.begin(), order.end(),
                                 [&](int x, int y) { return in_edges[x].size() > in_edges[y].size(); });
            }
            const int first = (b & 1) ? 64 : 0;
            const int n = std::max(0, std::min(64, (int)order.size() - first));
            for (int i = 0; i < 64; ++i) {
                lists[i].clear();
                if (i >= n) continue;
                for (uint32_t e : in_edges[order[first + i]]) lists[i].push_back({(int)((e / K) % NG), e});
            }
            const int steps = schedule_block(lists, n, member, seq);
            worst = std::max(worst, steps);
            wave_steps[(size_t)l * nblk + b] = steps;
            for (int lane = 0; lane < 64; ++lane) {
                const size_t slot = (size_t)l * npad + 64 * b + lane;
                lane_input[slot] = member[lane] < n ? order[first + member[lane]] : -1;
                for (int s = 0; s < dmax; ++s) {
                    uint32_t e = 0x80000000u;
                    if (s < (int)seq[lane].size()) {
                        e = seq[lane][s];
                        if (e & 0x80000000u) e = 0x80000000u | ((e & 0xffu) * K);
                    }
                    ent[slot * dmax + s] = e;
                }
            }
        }
    }
    return worst;
}

template <typename F>
int parallel_layers(int L, F f) {
    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    nth = std::min<unsigned>(nth, (unsigned)L);
    std::vector<std::thread> th;
    std::vector<int> worst(nth, 0);
    for (unsigned t = 0; t < nth; ++t) {
        const int l0 = (int)((int64_t)L * t / nth), l1 = (int)((int64_t)L * (t + 1) / nth);
        th.emplace_back([=, &worst, &f] { worst[t] = f(l0, l1); });
    }
    for (auto& x : th) x.join();
    return *std::max_element(worst.begin(), worst.end());
}

int build_schedule(const int32_t* idx, int N, int L, int dmax, uint32_t* ent, int32_t* lane_neuron,
                   int32_t* wave_steps) {
    return parallel_layers(L, [&](int l0, int l1) {
        return build_schedule_range(idx, N, l0, l1, dmax, ent, lane_neuron, wave_steps);
    });
}

int build_transposed_schedule(const int32_t* idx, int N, int L, int dmax, uint32_t* ent, int32_t* lane_input,
                              int32_t* wave_steps) {
    return parallel_layers(L, [&](int l0, int l1) {
        return build_transposed_range(idx, N, l0, l1, dmax, ent, lane_input, wave_steps);
    });
}

}  // namespace sdnn
