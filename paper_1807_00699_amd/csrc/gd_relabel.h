// Spin relabeling of one instance for the batched kernel's neighbour gathers
// (host code).
//
// In an item of T trajectories the amplitudes sit in LDS as rows of T
// consecutive words, row p at word p T, and one wave instruction gathers,
// for the G = 64 / T spins of G consecutive labels, the rows of their d-th
// neighbours.  The LDS has 64 banks of one word, so row p covers the banks of
// residue p mod G.  The model used here, which measurement favoured over
// whole 64-lane blocks, is that a 64-lane read is served in two passes of
// 32 lanes, i.e. of G / 2 rows, and that two different rows of one residue
// in a pass are read one after the other.  The relabeling permutes the spins so that in every
// block of `bs` consecutive labels (the rows of one pass: bs = G / 2) the
// d-th neighbours of the block's spins have different residues, for each d,
// as far as a local search gets.  Nothing numerical changes: a spin keeps its
// couplings in their list order, only the LDS row it lives in and the slot
// that updates it move.
//
// The search maximises the number of distinct (block, d, residue) triples
// (each duplicate is one more pass of an instruction): a conflicting triple
// is taken at random, and either the updated spin swaps labels with the best
// of a few random partners, or its neighbour with the best of a few spins of
// a residue the triple's block and d do not have yet; the swap is kept when
// it loses no triple.  Deterministic for a given seed.
#pragma once

#include <algorithm>
#include <cstdint>
#include <numeric>
#include <vector>

namespace gd {

struct RelabelResult {
    std::vector<int> label;     // label of spin i (a permutation of 0 .. n-1)
    long long conflicts0 = 0;   // duplicate triples before and after
    long long conflicts = 0;
};

// nb: [n][3] neighbour indices in list order (n: a missing coupling, which
// reads the zero row and is left out); g: the residue modulus (groups per
// gather instruction); bs: labels per block.
inline RelabelResult gather_relabel(int n, const std::vector<int> &nb, int g, int bs, uint64_t seed,
                                    long long max_moves) {
    RelabelResult res;
    res.label.resize(n);
    std::iota(res.label.begin(), res.label.end(), 0);
    if (g <= 1 || bs <= 1 || n < 2) return res;
    std::vector<int> &lab = res.label;
    std::vector<int> spin_at(n);
    std::iota(spin_at.begin(), spin_at.end(), 0);
    // who has spin j as its d-th neighbour: (x, d) pairs
    std::vector<int> roff(n + 1, 0), rx, rd;
    for (int x = 0; x < n; ++x)
        for (int d = 0; d < 3; ++d)
            if (nb[3 * x + d] < n) ++roff[nb[3 * x + d] + 1];
    for (int j = 0; j < n; ++j) roff[j + 1] += roff[j];
    rx.resize(roff[n]);
    rd.resize(roff[n]);
    {
        std::vector<int> fill(roff.begin(), roff.end() - 1);
        for (int x = 0; x < n; ++x)
            for (int d = 0; d < 3; ++d) {
                const int j = nb[3 * x + d];
                if (j < n) {
                    rx[fill[j]] = x;
                    rd[fill[j]] = d;
                    ++fill[j];
                }
            }
    }
    const int nblk = (n + bs - 1) / bs;
    std::vector<int> cnt((size_t)nblk * 3 * g, 0);
    long long contrib = 0, distinct = 0;
    auto entry = [&](int x, int d) -> int & {
        return cnt[((size_t)(lab[x] / bs) * 3 + d) * g + lab[nb[3 * x + d]] % g];
    };
    auto add = [&](int x, int d) {
        if (++entry(x, d) == 1) ++distinct;
    };
    auto sub = [&](int x, int d) {
        if (--entry(x, d) == 0) --distinct;
    };
    for (int x = 0; x < n; ++x)
        for (int d = 0; d < 3; ++d)
            if (nb[3 * x + d] < n) {
                add(x, d);
                ++contrib;
            }
    res.conflicts0 = contrib - distinct;
    // the contributions a swap of the labels of u and v changes: the d-th
    // neighbour terms of u and v and of every spin that has u or v as one
    int maxin = 0;
    for (int j = 0; j < n; ++j) maxin = std::max(maxin, roff[j + 1] - roff[j]);
    std::vector<std::pair<int, int>> aff(2 * (3 + maxin));
    int naff = 0;
    auto collect = [&](int u, int v) {
        naff = 0;
        auto put = [&](int x, int d) {
            for (int q = 0; q < naff; ++q)
                if (aff[q].first == x && aff[q].second == d) return;
            aff[naff++] = {x, d};
        };
        for (int s : {u, v}) {
            for (int d = 0; d < 3; ++d)
                if (nb[3 * s + d] < n) put(s, d);
            for (int q = roff[s]; q < roff[s + 1]; ++q) put(rx[q], rd[q]);
        }
    };
    auto swap_labels = [&](int u, int v) {
        std::swap(lab[u], lab[v]);
        spin_at[lab[u]] = u;
        spin_at[lab[v]] = v;
    };
    // distinct triples after swapping u and v (the swap is undone)
    auto try_swap = [&](int u, int v) {
        collect(u, v);
        for (int q = 0; q < naff; ++q) sub(aff[q].first, aff[q].second);
        swap_labels(u, v);
        for (int q = 0; q < naff; ++q) add(aff[q].first, aff[q].second);
        const long long after = distinct;
        for (int q = 0; q < naff; ++q) sub(aff[q].first, aff[q].second);
        swap_labels(u, v);
        for (int q = 0; q < naff; ++q) add(aff[q].first, aff[q].second);
        return after;
    };
    uint64_t st = seed * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
    auto rnd = [&](uint64_t m) {       // SplitMix64 step, reduced to [0, m)
        uint64_t z = (st += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        return (int)(z % m);
    };
    std::vector<std::pair<int, int>> bad;    // conflicting (spin, d)
    long long moves = 0;
    while (moves < max_moves && distinct < contrib) {
        bad.clear();
        for (int x = 0; x < n; ++x)
            for (int d = 0; d < 3; ++d)
                if (nb[3 * x + d] < n && entry(x, d) > 1) bad.push_back({x, d});
        const long long round = std::min<long long>((long long)bad.size() * 2, max_moves - moves);
        for (long long it = 0; it < round && distinct < contrib; ++it, ++moves) {
            const auto pick = bad[rnd(bad.size())];
            if (entry(pick.first, pick.second) <= 1) continue;     // resolved meanwhile
            const int x = pick.first, d = pick.second;
            // either move x to another block, or give its neighbour a
            // residue that no d-th neighbour of x's block has yet
            const bool move_nb = rnd(2) != 0;
            const int u = move_nb ? nb[3 * x + d] : x;
            int free_res[64], nfree = 0;
            if (move_nb) {
                const int *row = &cnt[((size_t)(lab[x] / bs) * 3 + d) * g];
                for (int c = 0; c < g && c < n; ++c)      // residues that some label has
                    if (row[c] == 0) free_res[nfree++] = c;
            }
            long long best = -1;
            int bv = -1;
            for (int c = 0; c < 6; ++c) {
                int v;
                if (nfree) {
                    // a random label of a free residue
                    const int r = free_res[rnd(nfree)];
                    const int blocks = (n - 1 - r) / g + 1;
                    v = spin_at[rnd(blocks) * g + r];
                } else {
                    v = rnd(n);
                }
                if (v == u) continue;
                const long long a = try_swap(u, v);
                if (a > best) {
                    best = a;
                    bv = v;
                }
            }
            if (bv >= 0 && best >= distinct) {
                collect(u, bv);
                for (int q = 0; q < naff; ++q) sub(aff[q].first, aff[q].second);
                swap_labels(u, bv);
                for (int q = 0; q < naff; ++q) add(aff[q].first, aff[q].second);
            }
        }
    }
    res.conflicts = contrib - distinct;
    return res;
}

}  // namespace gd
