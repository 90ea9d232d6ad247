// Create-time slot order of the one-row-tile kernel (host code).
//
// The kernel reads one activation row from LDS with 4-byte reads, one slot of
// one neuron per lane per step.  On gfx950 a wave's 4-byte LDS read is served in
// two halves of 32 lanes; a half whose lanes hit 32 distinct banks (word address
// mod 32) takes one pass, and a half with m lanes on its busiest bank takes m
// passes (measured with the LDS bank-conflict counter).  A neuron's 32 slots may
// be summed in any order, so for every half-wave block (32 neurons, one per lane)
// this file picks, per lane, the order in which it reads its slots.  Ascending
// slot order costs about 3.5 passes per read on random patterns.
//
// Construction for a block (32 lanes x 32 slots, bank of a slot = input id mod 32,
// d_b = slots of bank b over the block, sum d_b = 1024):
//  * a step in which every bank takes one lane uses all 32 banks, so at most
//    min_b d_b steps can be conflict-free; with K = max(max_b d_b - 32,
//    32 - min_b d_b) "double" steps (each bank at most two lanes, two passes) and
//    32 - K conflict-free steps the block costs 32 + K passes (about 45 instead of
//    about 112);
//  * phase 1 picks, by a max flow (lanes supply K slots, bank b demands
//    c_b = d_b - (32 - K)), which slots go to the double steps, leaving every bank
//    exactly 32 - K slots; splitting each bank into two halves of at most K edges
//    and colouring the edges with K colours (every bipartite multigraph of largest
//    degree D is D-edge-colourable, by alternating-path recolouring) gives the K
//    double steps;
//  * phase 2 colours the rest, a (32 - K)-regular bipartite multigraph, with
//    32 - K colours: each colour is a perfect matching, a conflict-free step.
// If the flow falls short, K grows by one; a partial block (fewer than 32 real
// neurons) is ordered greedily.
#include <algorithm>
#include <array>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <utility>
#include <vector>

#include "sdnn_internal.hpp"

namespace sdnn {

namespace {

constexpr int NB = 32;     // banks seen by a half-wave
constexpr int NL = 32;     // lanes of a half-wave block
constexpr int NS = K;      // slots per neuron

// Bipartite multigraph edge colouring with D <= 32 colours: left nodes nl, right
// nodes nr, every node of degree <= D.  Colour c of left node l goes to right node
// lc[l][c] (-1: free).
struct EdgeColouring {
    int nl = 0, nr = 0, D = 0;
    std::array<std::array<int8_t, 32>, 64> lc{}, rc{};
    std::array<uint32_t, 64> lm{}, rm{};   // used colours
    void init(int nl_, int nr_, int D_) {
        nl = nl_;
        nr = nr_;
        D = D_;
        for (auto& a : lc) a.fill(-1);
        for (auto& a : rc) a.fill(-1);
        lm.fill(0u);
        rm.fill(0u);
    }
    static int first_free(uint32_t m, int D) {
        const uint32_t f = ~m & (D >= 32 ? 0xffffffffu : ((1u << D) - 1u));
        return f ? __builtin_ctz(f) : -1;
    }
    void set(int l, int r, int c) {
        lc[l][c] = (int8_t)r;
        rc[r][c] = (int8_t)l;
        lm[l] |= 1u << c;
        rm[r] |= 1u << c;
    }
    void clear(int l, int r, int c) {
        lc[l][c] = -1;
        rc[r][c] = -1;
        lm[l] &= ~(1u << c);
        rm[r] &= ~(1u << c);
    }
    // colour one more edge (l, r); false if a node already has D edges
    bool add(int l, int r) {
        const int a = first_free(lm[l], D), b = first_free(rm[r], D);
        if (a < 0 || b < 0) return false;
        if (rc[r][a] >= 0) {
            // swap colours a and b on the path from r that alternates a, b, a, ...;
            // in a bipartite graph it cannot reach l, and afterwards a is free at r
            std::array<std::array<int, 3>, 130> path;
            int n = 0, cur = r, col = a;
            bool at_right = true;
            while (true) {
                if (at_right) {
                    const int nx = rc[cur][col];
                    if (nx < 0) break;
                    path[n++] = {nx, cur, col};
                    cur = nx;
                } else {
                    const int nx = lc[cur][col];
                    if (nx < 0) break;
                    path[n++] = {cur, nx, col};
                    cur = nx;
                }
                at_right = !at_right;
                col = col == a ? b : a;
            }
            for (int i = 0; i < n; ++i) clear(path[i][0], path[i][1], path[i][2]);
            for (int i = 0; i < n; ++i) set(path[i][0], path[i][1], path[i][2] == a ? b : a);
        }
        set(l, r, a);
        return true;
    }
};

// Max flow lanes (supply K each) -> banks (demand c[b]) over edge capacities
// cnt[l][b]; sel receives the flow.  Greedy start, then BFS augmenting paths.
bool select_double(const std::array<std::array<uint8_t, NB>, NL>& cnt, int Kd, const std::array<int, NB>& c,
                   std::array<std::array<uint8_t, NB>, NL>& sel) {
    for (auto& a : sel) a.fill(0);
    std::array<int, NL> supply;
    std::array<int, NB> demand = c;
    supply.fill(Kd);
    // greedy: each lane gives its units to the banks with the most unmet demand
    for (int l = 0; l < NL; ++l) {
        while (supply[l] > 0) {
            int best = -1;
            for (int b = 0; b < NB; ++b)
                if (cnt[l][b] > sel[l][b] && demand[b] > 0 && (best < 0 || demand[b] > demand[best])) best = b;
            if (best < 0) break;
            ++sel[l][best];
            --supply[l];
            --demand[best];
        }
    }
    // augment: source -> lane (supply) -> bank (cnt - sel) / bank -> lane (sel) -> sink (demand)
    while (true) {
        int total = 0;
        for (int b = 0; b < NB; ++b) total += demand[b];
        if (total == 0) return true;
        // BFS over lanes and banks from lanes with supply
        std::array<int, NL + NB> prev;
        prev.fill(-2);
        std::array<int, NL + NB> q;
        int qh = 0, qt = 0;
        for (int l = 0; l < NL; ++l)
            if (supply[l] > 0) {
                prev[l] = -1;
                q[qt++] = l;
            }
        int end = -1;
        while (qh < qt && end < 0) {
            const int u = q[qh++];
            if (u < NL) {
                for (int b = 0; b < NB; ++b)
                    if (prev[NL + b] == -2 && cnt[u][b] > sel[u][b]) {
                        prev[NL + b] = u;
                        if (demand[b] > 0) { end = NL + b; break; }
                        q[qt++] = NL + b;
                    }
            } else {
                const int b = u - NL;
                for (int l = 0; l < NL; ++l)
                    if (prev[l] == -2 && sel[l][b] > 0) {
                        prev[l] = u;
                        q[qt++] = l;
                    }
            }
        }
        if (end < 0) return false;
        // walk back: bank <- lane (add), lane <- bank (remove)
        int v = end;
        --demand[v - NL];
        while (true) {
            const int u = prev[v];
            if (v >= NL) {
                ++sel[u][v - NL];
            } else {
                if (u == -1) {
                    --supply[v];
                    break;
                }
                --sel[v][u - NL];
            }
            v = u;
        }
    }
}

// Greedy order for a partial block: at every step each lane takes a slot on a bank
// no other lane uses in that step if it has one (the heaviest such bank), else its
// heaviest bank.
void greedy_block(const std::array<std::array<uint8_t, NS>, NL>& bank, int nl,
                  std::array<std::array<uint8_t, NS>, NL>& perm) {
    std::array<std::array<bool, NS>, NL> done{};
    std::array<int, NB> left{};
    for (int l = 0; l < nl; ++l)
        for (int s = 0; s < NS; ++s) ++left[bank[l][s]];
    for (int st = 0; st < NS; ++st) {
        std::array<int, NB> used{};
        for (int l = 0; l < nl; ++l) {
            int pick = -1;
            for (int s = 0; s < NS; ++s) {
                if (done[l][s]) continue;
                const int b = bank[l][s];
                if (pick < 0) { pick = s; continue; }
                const int pb = bank[l][pick];
                const bool free_b = used[b] == 0, free_p = used[pb] == 0;
                if ((free_b && !free_p) || (free_b == free_p && left[b] > left[pb])) pick = s;
            }
            done[l][pick] = true;
            ++used[bank[l][pick]];
            --left[bank[l][pick]];
            perm[l][st] = (uint8_t)pick;
        }
    }
}

// Order of one half-wave block; returns its cost in LDS passes (sum over steps of
// the busiest bank's lane count).
int schedule_half(const std::array<std::array<uint8_t, NS>, NL>& bank, int nl,
                  std::array<std::array<uint8_t, NS>, NL>& perm) {
    if (nl < NL) {
        greedy_block(bank, nl, perm);
    } else {
        std::array<std::array<uint8_t, NB>, NL> cnt{};
        std::array<int, NB> d{};
        for (int l = 0; l < NL; ++l)
            for (int s = 0; s < NS; ++s) {
                ++cnt[l][bank[l][s]];
                ++d[bank[l][s]];
            }
        const int mx = *std::max_element(d.begin(), d.end()), mn = *std::min_element(d.begin(), d.end());
        int Kd = std::max(0, std::max(mx - NS, NS - mn));
        bool ok = false;
        std::array<std::array<uint8_t, NB>, NL> sel{};
        EdgeColouring ec;
        std::array<int, NB> c{};
        for (; Kd <= NS && !ok; ++Kd) {
            const int R2 = NS - Kd;
            bool fits = true;
            for (int b = 0; b < NB; ++b) {
                c[b] = d[b] - R2;
                if (c[b] < 0 || c[b] > 2 * Kd) fits = false;
            }
            if (!fits || !select_double(cnt, Kd, c, sel)) continue;
            ok = true;
            std::array<std::array<std::vector<uint8_t>, NB>, NL> pool;
            for (int l = 0; l < NL; ++l)
                for (int s = 0; s < NS; ++s) pool[l][bank[l][s]].push_back((uint8_t)s);
            // phase 1: each bank split into two right nodes of at most Kd edges
            if (Kd > 0) {
                ec.init(NL, 2 * NB, Kd);
                std::array<int, NB> units{};
                for (int l = 0; l < NL && ok; ++l)
                    for (int b = 0; b < NB && ok; ++b)
                        for (int u = 0; u < sel[l][b]; ++u) ok = ec.add(l, 2 * b + (units[b]++ & 1));
                for (int l = 0; l < NL && ok; ++l)
                    for (int st = 0; st < Kd; ++st) {
                        const int b = ec.lc[l][st] >> 1;
                        perm[l][st] = pool[l][b].back();
                        pool[l][b].pop_back();
                    }
            }
            // phase 2: the (32 - Kd)-regular rest, one perfect matching per colour
            if (ok && R2 > 0) {
                ec.init(NL, NB, R2);
                for (int l = 0; l < NL && ok; ++l)
                    for (int b = 0; b < NB && ok; ++b)
                        for (size_t u = 0; u < pool[l][b].size() && ok; ++u) ok = ec.add(l, b);
                for (int l = 0; l < NL && ok; ++l)
                    for (int st = 0; st < R2; ++st) {
                        const int b = ec.lc[l][st];
                        perm[l][Kd + st] = pool[l][b].back();
                        pool[l][b].pop_back();
                    }
            }
        }
        if (!ok) greedy_block(bank, nl, perm);
    }
    int cost = 0;
    for (int st = 0; st < NS; ++st) {
        std::array<int, NB> m{};
        int w = 0;
        for (int l = 0; l < nl; ++l) w = std::max(w, ++m[bank[l][perm[l][st]]]);
        cost += w;
    }
    return cost;
}

}  // namespace

// Slot order of the one-row-tile kernel for layers [0, L): perm[l][j][step] = the
// slot neuron j reads at that step.  The kernel's half-wave blocks are 32
// consecutive neurons (lane j % 32 of a half-wave), so blocks are aligned at
// multiples of 32.  Returns the summed cost in LDS passes (for tests and logs).
int64_t build_row_schedule(const int32_t* idx, int N, int L, uint8_t* perm) {
    const int nblk = (N + NL - 1) / NL;
    const int64_t total = (int64_t)L * nblk;
    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    nth = (unsigned)std::max<int64_t>(1, std::min<int64_t>(nth, total));
    std::vector<int64_t> cost(nth, 0);
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nth; ++t) {
        th.emplace_back([=, &cost] {
            std::array<std::array<uint8_t, NS>, NL> bank{}, pm{};
            for (int64_t i = total * t / nth; i < total * (t + 1) / nth; ++i) {
                const int l = (int)(i / nblk), blk = (int)(i % nblk);
                const int j0 = blk * NL, nl = std::min(NL, N - j0);
                const int32_t* il = idx + ((size_t)l * N + j0) * NS;
                for (int x = 0; x < nl; ++x)
                    for (int s = 0; s < NS; ++s) bank[x][s] = (uint8_t)((uint32_t)il[x * NS + s] % NB);
                cost[t] += schedule_half(bank, nl, pm);
                uint8_t* out = perm + ((size_t)l * N + j0) * NS;
                for (int x = 0; x < nl; ++x) std::memcpy(out + x * NS, pm[x].data(), NS);
            }
        });
    }
    for (auto& x : th) x.join();
    int64_t sum = 0;
    for (int64_t v : cost) sum += v;
    return sum;
}

// ---------------------------------------------------------------- neuron pairs
// Neuron pairs of the chunked one-row-tile kernel (sdnn_rowc.hip).  A lane holds
// two neurons in 64 register positions, 64 / C per chunk of the row; a pair whose
// slots in a chunk exceed the chunk's positions keeps the excess in a per-part LDS
// list, so pairs should complement each other: a neuron with many slots in some
// chunks goes with one that has few there.  Per part (2048 neurons):
//  * C = 2: the count in chunk 0 decides (chunk 1 has the rest), so pairing the
//    i-th smallest count with the i-th largest balances every pair;
//  * C = 4: neurons in order of decreasing imbalance (sum over chunks of
//    |count - 8|) each take the unpaired partner with the least overflow (then
//    the least squared deviation from 16 per chunk), searched among the count
//    vectors within distance 2 (per chunk) of the ideal complement 16 - count,
//    nearest first, or among all unpaired neurons when none is that close.
// Then the part's pairs are put in order of decreasing overflow: a wave runs its
// overflow loop as often as its busiest lane needs, so pairs with excess share
// waves (for random C = 4 patterns three quarters of the loop trips of the
// pairing's own order, which puts the most unbalanced neurons first).
namespace {

uint32_t cnt_of(uint32_t v, int c) { return (v >> (8 * c)) & 0xffu; }

// overflow entries and squared imbalance of a pair
std::pair<int, int> pair_cost(uint32_t a, uint32_t b, int C) {
    const int PC = 64 / C;
    int ov = 0, dv = 0;
    for (int c = 0; c < C; ++c) {
        const int t = (int)(cnt_of(a, c) + cnt_of(b, c));
        ov += t > PC ? t - PC : 0;
        dv += (t - PC) * (t - PC);
    }
    return {ov, dv};
}

struct PairBuckets {
    static constexpr int E = 33;            // count values 0..32
    std::vector<std::vector<int>> bucket = std::vector<std::vector<int>>(E * E * E);
    std::vector<int> where;                 // position of a neuron in its bucket
    std::vector<int> touched;
    static int key(uint32_t v) { return (int)(cnt_of(v, 0) * E * E + cnt_of(v, 1) * E + cnt_of(v, 2)); }
    void add(int j, uint32_t v) {
        auto& b = bucket[key(v)];
        if (b.empty()) touched.push_back(key(v));
        where[j] = (int)b.size();
        b.push_back(j);
    }
    void remove(int j, uint32_t v) {
        auto& b = bucket[key(v)];
        const int at = where[j], last = b.back();
        b[at] = last;
        where[last] = at;
        b.pop_back();
    }
    void clear() {
        for (int k : touched) bucket[k].clear();
        touched.clear();
    }
};

// pairs of one part: out[lane] = first | second << 16 (neurons within the part);
// returns the part's overflow entries
int pair_part(const uint32_t* cnt, int n, int C, uint32_t* out, PairBuckets& pb) {
    std::vector<int> order(n);
    for (int j = 0; j < n; ++j) order[j] = j;
    int total = 0, lanes = 0;
    if (C == 2) {
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cnt_of(cnt[x], 0) < cnt_of(cnt[y], 0); });
        for (int i = 0; i < n / 2; ++i) {
            const int a = order[i], b = order[n - 1 - i];
            out[lanes++] = (uint32_t)a | ((uint32_t)b << 16);
            total += pair_cost(cnt[a], cnt[b], C).first;
        }
        return total;
    }
    const int PC = 64 / C;
    auto imbalance = [&](int j) {
        int e = 0;
        for (int c = 0; c < C; ++c) e += std::abs((int)cnt_of(cnt[j], c) - PC / 2);
        return e;
    };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return imbalance(x) > imbalance(y); });
    pb.where.assign(n, 0);
    std::vector<char> used(n, 0);
    for (int j = 0; j < n; ++j) pb.add(j, cnt[j]);
    for (int i : order) {
        if (used[i]) continue;
        used[i] = 1;
        pb.remove(i, cnt[i]);
        const int u0 = PC - (int)cnt_of(cnt[i], 0), u1 = PC - (int)cnt_of(cnt[i], 1), u2 = PC - (int)cnt_of(cnt[i], 2);
        int best = -1;
        std::pair<int, int> bc{1 << 30, 1 << 30};
        for (int r = 0; r <= 2; ++r) {
            for (int d0 = -r; d0 <= r; ++d0)
                for (int d1 = -r; d1 <= r; ++d1)
                    for (int d2 = -r; d2 <= r; ++d2) {
                        if (std::max(std::abs(d0), std::max(std::abs(d1), std::abs(d2))) != r) continue;
                        const int v0 = u0 + d0, v1 = u1 + d1, v2 = u2 + d2;
                        if (v0 < 0 || v1 < 0 || v2 < 0 || v0 > 32 || v1 > 32 || v2 > 32) continue;
                        const auto& b = pb.bucket[v0 * PairBuckets::E * PairBuckets::E + v1 * PairBuckets::E + v2];
                        if (b.empty()) continue;
                        const int j = b.back();
                        const auto c = pair_cost(cnt[i], cnt[j], C);
                        if (c < bc) { bc = c; best = j; }
                    }
            if (best >= 0 && bc.first == 0) break;
        }
        if (best < 0) {
            for (int j = 0; j < n; ++j)
                if (!used[j]) {
                    const auto c = pair_cost(cnt[i], cnt[j], C);
                    if (c < bc) { bc = c; best = j; }
                }
        }
        if (best < 0) break;                      // (n is even: never)
        used[best] = 1;
        pb.remove(best, cnt[best]);
        out[lanes++] = (uint32_t)i | ((uint32_t)best << 16);
        total += bc.first;
    }
    pb.clear();
    return total;
}

}  // namespace

int build_rowc_pairs(const uint32_t* counts, int N, int L, int C, uint32_t* pairs) {
    if (N % ROW_PART != 0 || (C != 2 && C != 4) || L < 1) return -1;
    const int G = N / ROW_PART;
    const int64_t total = (int64_t)L * G;
    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    nth = (unsigned)std::max<int64_t>(1, std::min<int64_t>(nth, total));
    std::vector<int> worst(nth, 0);
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nth; ++t) {
        th.emplace_back([=, &worst] {
            PairBuckets pb;
            for (int64_t i = total * t / nth; i < total * (t + 1) / nth; ++i) {
                const int l = (int)(i / G), p = (int)(i % G);
                const uint32_t* cnt = counts + (size_t)l * N + (size_t)p * ROW_PART;
                uint32_t* out = pairs + (size_t)l * (N / 2) + (size_t)p * (ROW_PART / 2);
                worst[t] = std::max(worst[t], pair_part(cnt, ROW_PART, C, out, pb));
                auto excess = [cnt, C](uint32_t pr) { return pair_cost(cnt[pr & 0xffffu], cnt[pr >> 16], C).first; };
                std::stable_sort(out, out + ROW_PART / 2, [&](uint32_t x, uint32_t y) { return excess(x) > excess(y); });
            }
        });
    }
    for (auto& x : th) x.join();
    return *std::max_element(worst.begin(), worst.end());
}

}  // namespace sdnn
