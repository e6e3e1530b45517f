// Reads "n g bs seed moves" and n lines of three neighbour indices from
// stdin, runs gd::gather_relabel and prints "conflicts0 conflicts" and the n
// labels.  Host code; compiled by the test that uses it.
#include "gd_relabel.h"

#include <cstdio>

int main() {
    int n, g, bs;
    unsigned long long seed;
    long long moves;
    if (std::scanf("%d %d %d %llu %lld", &n, &g, &bs, &seed, &moves) != 5) return 2;
    std::vector<int> nb((size_t)3 * n);
    for (auto &v : nb)
        if (std::scanf("%d", &v) != 1) return 2;
    const gd::RelabelResult r = gd::gather_relabel(n, nb, g, bs, seed, moves);
    std::printf("%lld %lld\n", r.conflicts0, r.conflicts);
    for (int v : r.label) std::printf("%d\n", v);
    return 0;
}
