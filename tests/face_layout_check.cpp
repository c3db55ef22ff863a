// Host check of the blocked face-plane layout (FacePlane in rt_internal.h): every
// vertex of a slot has its own position inside the slot, and in a simulated slot
// the halo a tile reads (its 9 x 9 incoming face: the 8 x 8 interior, the row at
// b = g0b - 1 and the column at a = g0a - 1) holds the vertices that the tiles beside
// and below it and the ghost fill wrote, addressed as the sweep kernels address them.
#include "../paper_1201_2222_amd/csrc/rt_internal.h"

#include <cstdio>
#include <vector>

using rtsc::FacePlane;

static int fails = 0;
#define CHECK(c, ...)                       \
    do {                                    \
        if (!(c)) {                         \
            if (fails++ < 20) {             \
                std::printf(__VA_ARGS__);   \
                std::printf("\n");          \
            }                               \
        }                                   \
    } while (0)

static void check(int na, int nb, int slot_index)
{
    const FacePlane F(na, nb);
    const long S = (long)F.slot();
    const int T = rtsc::kTile;
    auto id = [&](int a, int b) { return (a + 1) * (nb + 1) + (b + 1); };
    std::vector<int> mem(S, -1);
    auto put = [&](long pos, int v) {
        CHECK(pos >= 0 && pos < S, "na %d nb %d: write at %ld outside the slot of %ld", na, nb, pos, S);
        if (pos >= 0 && pos < S) mem[pos] = v;
    };
    // distinct positions for every vertex
    std::vector<int> seen(S, 0);
    for (int b = -1; b < nb; ++b)
        for (int a = -1; a < na; ++a) {
            const long p = F.at(a, b);
            CHECK(p >= 0 && p < S, "na %d nb %d: vertex (%d, %d) at %ld outside %ld", na, nb, a, b, p, S);
            if (p >= 0 && p < S) {
                CHECK(seen[p] == 0, "na %d nb %d: vertex (%d, %d) shares position %ld", na, nb, a, b, p);
                seen[p] = 1;
            }
            if (a >= 0 && b >= 0 && (a & (T - 1)) == T - 1) {
                const long c = F.col(a, b);
                CHECK(c >= 0 && c < S && !seen[c], "na %d nb %d: copy of (%d, %d) at %ld", na, nb, a, b, c);
                if (c >= 0 && c < S) seen[c] = 1;
            }
        }
    // fill the slot: slot 0 entirely by the ghost fill (with the copies), later slots
    // by the tiles of the previous layer (8 x 8 each, copies on a full block's last
    // column) and the ghost fill (row b = -1, column a = -1)
    const int nta = (na + T - 1) / T, ntb = (nb + T - 1) / T;
    for (int b = -1; b < nb; ++b)
        for (int a = -1; a < na; ++a) {
            const bool ghost = a < 0 || b < 0;
            if (slot_index > 0 && !ghost) continue;
            put(F.at(a, b), id(a, b));
            if (!ghost && (a & (T - 1)) == T - 1) put(F.col(a, b), id(a, b));
        }
    if (slot_index > 0)
        for (int tb = 0; tb < ntb; ++tb)
            for (int ta = 0; ta < nta; ++ta)
                for (int w = 0; w < T; ++w)
                    for (int u = 0; u < T; ++u) {
                        const int a = ta * T + u, b = tb * T + w;
                        if (a >= na || b >= nb) continue;
                        put(F.at(a, b), id(a, b));
                        if (u == T - 1) put(F.col(a, b), id(a, b));
                    }
    // every tile's reads
    for (int tb = 0; tb < ntb; ++tb)
        for (int ta = 0; ta < nta; ++ta) {
            const int g0a = ta * T, g0b = tb * T;
            const int ea = na - g0a < T ? na - g0a : T, eb = nb - g0b < T ? nb - g0b : T;
            for (int w = 0; w < T; ++w)
                for (int u = 0; u < T; ++u) {   // the kernels' forms: block base + lane
                    CHECK(F.blk(ta, tb) + 8 * w + u == F.at(g0a + u, g0b + w), "na %d nb %d: block base (%d, %d)", na,
                          nb, ta, tb);
                    if (u == T - 1)
                        CHECK(F.colblk(ta, tb) + w == F.col(g0a + u, g0b + w), "na %d nb %d: column base (%d, %d)", na,
                              nb, ta, tb);
                }
            for (int w = 0; w < eb; ++w)
                for (int u = 0; u < ea; ++u) {
                    const long p = F.blk(ta, tb) + 8 * w + u;
                    CHECK(p >= 0 && p < S && mem[p] == id(g0a + u, g0b + w), "na %d nb %d slot %d: interior (%d, %d)",
                          na, nb, slot_index, g0a + u, g0b + w);
                }
            for (int j = 0; j <= ea; ++j) {   // the row at b = g0b - 1, a = g0a - 1 .. g0a + ea - 1
                const long p = F.at(g0a + j - 1, g0b - 1);
                CHECK(p >= 0 && p < S && mem[p] == id(g0a + j - 1, g0b - 1), "na %d nb %d slot %d: row (%d, %d)", na,
                      nb, slot_index, g0a + j - 1, g0b - 1);
            }
            for (int j = 0; j < eb; ++j) {    // the column at a = g0a - 1, b = g0b .. g0b + eb - 1
                const long p = ta > 0 ? F.colblk(ta - 1, tb) + j : F.at(-1, g0b + j);
                CHECK(p >= 0 && p < S && mem[p] == id(g0a - 1, g0b + j), "na %d nb %d slot %d: column (%d, %d)", na,
                      nb, slot_index, g0a - 1, g0b + j);
            }
        }
}

int main()
{
    const int sizes[][2] = {{1, 1}, {1, 20}, {8, 8}, {9, 17}, {13, 11}, {16, 24}, {19, 13}, {40, 7}, {64, 64},
                            {127, 3}, {128, 128}, {192, 192}};
    for (const auto &s : sizes)
        for (int slot = 0; slot < 2; ++slot) check(s[0], s[1], slot);
    std::printf("%s\n", fails ? "FAIL" : "OK");
    return fails ? 1 : 0;
}
