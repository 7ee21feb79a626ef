// CPU check of the Schwarz block tables that the field set-up copies to the
// device (block_tables.h).  Every entry is compared with what the global site
// coordinates give, computed here without the builder's code: in-block
// neighbours, the face lists of every direction, the site across the face
// that feeds each entry, the neighbouring block the entry is read from, the
// antiperiodic time-boundary sign, and the colour-major block layout.
// Usage: host_tables_check L0 L1 L2 L3 b0 b1 b2 b3 bc_t; exit status 0 when
// every check holds.  Built with the address and undefined-behaviour
// sanitizers by tests/test_host_tables.py.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "block_tables.h"

namespace {

int L[4], b[4], nb[4], bc;
long errors = 0;

void fail(const char *what, long a, long c) {
    if (errors++ < 10) std::fprintf(stderr, "mismatch: %s (%ld, %ld)\n", what, a, c);
}

// lexicographic index over extents e (last axis fastest)
int lex(const int c[4], const int e[4]) { return ((c[0] * e[1] + c[1]) * e[2] + c[2]) * e[3] + c[3]; }
void unlex(int i, const int e[4], int c[4]) {
    for (int m = 3; m >= 0; --m) {
        c[m] = i % e[m];
        i /= e[m];
    }
}
int parity(const int c[4]) { return (c[0] + c[1] + c[2] + c[3]) & 1; }

}  // namespace

int main(int argc, char **argv) {
    if (argc != 10) {
        std::fprintf(stderr, "usage: %s L0 L1 L2 L3 b0 b1 b2 b3 bc_t\n", argv[0]);
        return 2;
    }
    for (int m = 0; m < 4; ++m) {
        L[m] = std::atoi(argv[1 + m]);
        b[m] = std::atoi(argv[5 + m]);
        nb[m] = L[m] / b[m];
    }
    bc = std::atoi(argv[9]);
    dfl::BlockTables t;
    dfl::build_block_tables(b, nb, bc, t);
    const int Vb = b[0] * b[1] * b[2] * b[3], Vbh = Vb / 2, Nb = nb[0] * nb[1] * nb[2] * nb[3];

    // the colour-major layout: a bijection, colour 0 (even block-coordinate
    // sum) in the first half, each colour in lexicographic order
    std::vector<int> seen(Nb, 0);
    int rank[2] = {0, 0};
    for (int Bl = 0; Bl < Nb; ++Bl) {
        int cb[4];
        unlex(Bl, nb, cb);
        const int col = parity(cb), want = col * (Nb / 2) + rank[col]++;
        if (t.bord[Bl] != want) fail("block place", Bl, t.bord[Bl]);
        if (t.bord[Bl] >= 0 && t.bord[Bl] < Nb) seen[t.bord[Bl]]++;
    }
    for (int p = 0; p < Nb; ++p)
        if (seen[p] != 1) fail("block layout is not a bijection", p, seen[p]);
    std::vector<int> block_at(Nb);
    for (int Bl = 0; Bl < Nb; ++Bl) block_at[t.bord[Bl]] = Bl;

    // in-block neighbours
    for (int l = 0; l < Vb; ++l) {
        int c[4];
        unlex(l, b, c);
        for (int mu = 0; mu < 4; ++mu)
            for (int d = 0; d < 2; ++d) {
                int cc[4] = {c[0], c[1], c[2], c[3]};
                cc[mu] += d == 0 ? 1 : -1;
                const bool inside = cc[mu] >= 0 && cc[mu] < b[mu];
                const int want = inside ? lex(cc, b) / 2 : -1;
                const int got = t.lnb[((size_t)parity(c) * Vbh + l / 2) * 8 + 2 * mu + d];
                if (got != want) fail("in-block neighbour", l, 2 * mu + d);
            }
    }

    // face lists: every face site exactly once, in (d, parity, j) order
    for (int mu = 0; mu < 4; ++mu) {
        std::vector<int> count(2 * Vb, 0);
        for (int k = 0; k < t.nface[mu]; ++k) {
            const int ent = t.fl[(size_t)mu * t.face_cap + k];
            const int par = ent >> 30, d = (ent >> 29) & 1, j = ent & 0x1fffffff;
            if (j < 0 || j >= Vbh) {
                fail("face entry out of range", mu, k);
                continue;
            }
            count[d * Vb + par * Vbh + j]++;
            if (k > 0) {
                const int prev = t.fl[(size_t)mu * t.face_cap + k - 1];
                const int pd = (prev >> 29) & 1, pp = prev >> 30, pj = prev & 0x1fffffff;
                if (pd > d || (pd == d && (pp > par || (pp == par && pj >= j)))) fail("face order", mu, k);
            }
        }
        for (int l = 0; l < Vb; ++l) {
            int c[4];
            unlex(l, b, c);
            for (int d = 0; d < 2; ++d) {
                const bool on = c[mu] == (d == 0 ? b[mu] - 1 : 0);
                if (count[d * Vb + parity(c) * Vbh + l / 2] != (on ? 1 : 0)) fail("face membership", mu, l);
            }
        }
    }

    // every entry of every block: the site across the face, its block, the sign
    for (int Bl = 0; Bl < Nb; ++Bl) {
        int cb[4];
        unlex(Bl, nb, cb);
        for (int mu = 0; mu < 4; ++mu)
            for (int k = 0; k < t.nface[mu]; ++k) {
                const int ent = t.fl[(size_t)mu * t.face_cap + k];
                const int par = ent >> 30, d = (ent >> 29) & 1, j = ent & 0x1fffffff;
                // the reader's site x: local index 2j or 2j + 1, whichever has the parity
                int cx[4], l = 2 * j;
                unlex(l, b, cx);
                if (parity(cx) != par) unlex(++l, b, cx);
                int x[4], y[4];
                for (int m = 0; m < 4; ++m) x[m] = cb[m] * b[m] + cx[m];
                for (int m = 0; m < 4; ++m) y[m] = x[m];
                y[mu] += d == 0 ? 1 : -1;
                const bool wrap = y[mu] < 0 || y[mu] >= L[mu];
                y[mu] = (y[mu] + L[mu]) % L[mu];
                int cby[4], cy[4];
                for (int m = 0; m < 4; ++m) {
                    cby[m] = y[m] / b[m];
                    cy[m] = y[m] % b[m];
                }
                const int writer = t.bord[lex(cby, nb)];
                const int src = t.fsrc[(size_t)mu * t.face_cap + k];
                if (src != ((parity(cy) << 30) | (lex(cy, b) / 2))) fail("face source", Bl, mu * 100000 + k);
                const int nbv = t.fnb[(size_t)writer * 8 + 2 * mu + d];
                if ((nbv & 0x7fffffff) != t.bord[Bl]) fail("face neighbour block", Bl, mu);
                const bool sign = (unsigned)nbv >> 31;
                if (sign != (mu == 0 && wrap && bc == -1)) fail("boundary sign", Bl, mu);
                if (block_at[writer] != lex(cby, nb)) fail("writer block", Bl, mu);
            }
    }
    long tot = 0;
    for (int mu = 0; mu < 4; ++mu) tot += t.nface[mu];
    if (tot != t.nface_tot) fail("face total", tot, t.nface_tot);
    std::printf("lattice %dx%dx%dx%d blocks %dx%dx%dx%d bc %d: %d blocks, %d face entries per block, %ld mismatches\n",
                L[0], L[1], L[2], L[3], b[0], b[1], b[2], b[3], bc, Nb, t.nface_tot, errors);
    return errors ? 1 : 0;
}
