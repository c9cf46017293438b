// Host check of the bit-parallel Levenshtein recurrences of the device code
// (myers_distance for 1..4 words, myers_banded for cutoffs up to 63) against
// the textbook dynamic programme D[i][j] = min(D[i-1][j] + 1, D[i][j-1] + 1,
// D[i-1][j-1] + [a_i != b_j]).  Contract checked: the exact distance when it
// is <= cutoff, some value > cutoff otherwise.  Strings: random, and mutated
// copies (substitutions, insertions, deletions) so that both sides of the
// cutoff occur; lengths 0..255; 2- and 4-letter alphabets.
// usage: myers_host <seed> <cases>; prints "ok <cases>" or the first mismatch.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "../paper_2404_00966_amd/csrc/dev_common.h"

namespace {

int dp(const std::vector<int> &a, const std::vector<int> &b)
{
    const int m = (int)a.size(), n = (int)b.size();
    std::vector<int> prev(n + 1), cur(n + 1);
    for (int j = 0; j <= n; j++) prev[j] = j;
    for (int i = 1; i <= m; i++) {
        cur[0] = i;
        for (int j = 1; j <= n; j++)
            cur[j] = std::min({prev[j] + 1, cur[j - 1] + 1, prev[j - 1] + (a[i - 1] != b[j - 1] ? 1 : 0)});
        std::swap(prev, cur);
    }
    return prev[n];
}

struct Codes {
    int operator[](int c) const { return c; }
};

}  // namespace

int main(int argc, char **argv)
{
    const unsigned seed = argc > 1 ? (unsigned)std::atoi(argv[1]) : 1u;
    const long cases = argc > 2 ? std::atol(argv[2]) : 100000;
    std::mt19937 g(seed);
    for (long it = 0; it < cases; it++) {
        const int sigma = it % 7 == 0 ? 2 : 4;
        const int m = (int)(g() % 256);
        std::vector<int> a(m), b;
        for (int &x : a) x = (int)(g() % sigma);
        if (it % 3 != 0) {
            b = a;
            const int edits = (int)(g() % (it % 5 == 0 ? 80 : 20));
            for (int e = 0; e < edits; e++) {
                const int kind = (int)(g() % 3);
                const int p = (int)(g() % (b.size() + 1));
                if (kind == 0 && p < (int)b.size()) b[p] = (int)(g() % sigma);
                else if (kind == 1 && b.size() < 255) b.insert(b.begin() + p, (int)(g() % sigma));
                else if (kind == 2 && p < (int)b.size()) b.erase(b.begin() + p);
            }
        } else {
            b.resize(g() % 256);
            for (int &x : b) x = (int)(g() % sigma);
        }
        const int n = (int)b.size();
        std::vector<uint64_t> peq(4 * 4, 0ull);
        for (int i = 0; i < m; i++) peq[a[i] * 4 + (i >> 6)] |= 1ull << (i & 63);
        std::vector<uint8_t> text(n);
        for (int j = 0; j < n; j++) text[j] = (uint8_t)b[j];
        const int d = dp(a, b);
        const int words = std::max(1, (m + 63) / 64);
        const int cut_full = it % 4 == 0 ? (1 << 30) : (int)(g() % 100);
        int full;
        switch (words) {
        case 1: full = gts::dev::myers_distance<1>(peq.data(), m, text.data(), n, cut_full, Codes{}); break;
        case 2: full = gts::dev::myers_distance<2>(peq.data(), m, text.data(), n, cut_full, Codes{}); break;
        case 3: full = gts::dev::myers_distance<3>(peq.data(), m, text.data(), n, cut_full, Codes{}); break;
        default: full = gts::dev::myers_distance<4>(peq.data(), m, text.data(), n, cut_full, Codes{}); break;
        }
        const int cut_band = (int)(g() % 64);
        const int nw = it % 2 ? 4 : words;   // tables of 4 words, or of the pattern's own word count
        const int band = gts::dev::myers_banded(peq.data(), nw, m, text.data(), n, cut_band, Codes{});
        const bool ok_full = d <= cut_full ? full == d : full > cut_full;
        const bool ok_band = d <= cut_band ? band == d : band > cut_band;
        if (!ok_full || !ok_band) {
            std::printf("mismatch case %ld: m=%d n=%d d=%d full(cut %d)=%d banded(cut %d)=%d\n", it, m, n, d,
                        cut_full, full, cut_band, band);
            return 1;
        }
    }
    std::printf("ok %ld\n", cases);
    return 0;
}
