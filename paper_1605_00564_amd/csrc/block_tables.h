// Host-side tables of the Schwarz block decomposition: the in-block
// neighbours of the block shape, the per-direction lists of the sites on a
// block's faces with the site across the face that feeds each of them, the
// colour-major order of the blocks and the neighbouring blocks of the face
// exchange.  Plain C++ (no device code): the field set-up copies the tables
// to the device, and a CPU test builds and checks them.
#pragma once

#include <algorithm>
#include <vector>

namespace dfl {

struct BlockTables {
    std::vector<short> lnb;   // [2 parity][Vbh][8]: in-block neighbour (local j) in direction 2 mu + d, or -1
    std::vector<int> fl;      // [4][face_cap]: face entries (parity << 30 | d << 29 | j), nface[mu] used
    std::vector<int> fsrc;    // [4][face_cap]: the site across the face feeding each entry (parity << 30 | j)
    std::vector<int> bord;    // [Nb]: block in lexicographic order -> its place in the colour-major layout
    std::vector<int> fnb;     // [Nb][8] by place: the block fed through entries of kind 2 mu + d, bit 31 =
                              // the hop crosses the antiperiodic time boundary
    int nface[4] = {0, 0, 0, 0};
    int face_cap = 0;
    int nface_tot = 0;
};

// b: block extents (even); nb: blocks per direction (even); bc_t: +1 or -1.
// Sites of a block are numbered lexicographically (last axis fastest) by l;
// j = l >> 1 enumerates each parity half.
inline void build_block_tables(const int b[4], const int nb[4], int bc_t, BlockTables &t) {
    const int Vb = b[0] * b[1] * b[2] * b[3], Vbh = Vb / 2, Nb = nb[0] * nb[1] * nb[2] * nb[3];
    auto coords = [&](int l, int c[4]) {
        int r = l;
        for (int m = 3; m >= 0; --m) {
            c[m] = r % b[m];
            r /= b[m];
        }
    };
    // in-block neighbours (parity of l's coordinates, j = l >> 1)
    t.lnb.assign((size_t)16 * Vbh, -1);
    for (int l = 0; l < Vb; ++l) {
        int c[4];
        coords(l, c);
        const int p = (c[0] + c[1] + c[2] + c[3]) & 1;
        for (int mu = 0; mu < 4; ++mu)
            for (int d = 0; d < 2; ++d) {
                int cc[4] = {c[0], c[1], c[2], c[3]};
                cc[mu] += d == 0 ? 1 : -1;
                if (cc[mu] < 0 || cc[mu] >= b[mu]) continue;
                int l2 = 0;
                for (int m = 0; m < 4; ++m) l2 = l2 * b[m] + cc[m];
                t.lnb[((size_t)p * Vbh + (l >> 1)) * 8 + 2 * mu + d] = (short)(l2 >> 1);
            }
    }
    // hops that leave a block, grouped by direction mu: the forward-face
    // sites (both parities) first, then the backward-face ones; the two
    // faces of one mu are disjoint because block extents are at least 2
    std::vector<int> face[4];
    for (int mu = 0; mu < 4; ++mu)
        for (int d = 0; d < 2; ++d)
            for (int l = 0; l < Vb; ++l) {
                int c[4];
                coords(l, c);
                if (c[mu] != (d == 0 ? b[mu] - 1 : 0)) continue;
                const int p = (c[0] + c[1] + c[2] + c[3]) & 1;
                face[mu].push_back((p << 30) | (d << 29) | (l >> 1));
            }
    // within a face, parity-major and ascending j: consecutive lanes then
    // read consecutive exchange-buffer rows of one parity (no bank conflicts)
    for (int mu = 0; mu < 4; ++mu)
        std::sort(face[mu].begin(), face[mu].end(), [](int a, int c) {
            const int da = (a >> 29) & 1, dc = (c >> 29) & 1;
            return da != dc ? da < dc : a < c;
        });
    t.face_cap = 0;
    t.nface_tot = 0;
    for (int mu = 0; mu < 4; ++mu) {
        t.nface[mu] = (int)face[mu].size();
        t.face_cap = std::max(t.face_cap, t.nface[mu]);
        t.nface_tot += t.nface[mu];
    }
    t.fl.assign((size_t)4 * t.face_cap, 0);
    for (int mu = 0; mu < 4; ++mu) std::copy(face[mu].begin(), face[mu].end(), t.fl.begin() + (size_t)mu * t.face_cap);
    // the source of each face entry: x on the forward face (d = 0) is fed by
    // x + mu, the site with c_mu = 0 in the next block; x on the backward
    // face by x - mu, the site with c_mu = b_mu - 1 in the previous block
    t.fsrc.assign((size_t)4 * t.face_cap, 0);
    for (int mu = 0; mu < 4; ++mu)
        for (int k = 0; k < t.nface[mu]; ++k) {
            const int ent = face[mu][k], par = ent >> 30, d = (ent >> 29) & 1, j = ent & 0x1fffffff;
            int c[4], l = -1;
            for (int cand = 2 * j; cand <= 2 * j + 1 && l < 0; ++cand) {
                coords(cand, c);
                if (((c[0] + c[1] + c[2] + c[3]) & 1) == par) l = cand;
            }
            coords(l, c);
            c[mu] = d == 0 ? 0 : b[mu] - 1;
            int l2 = 0, sum = 0;
            for (int m = 0; m < 4; ++m) {
                l2 = l2 * b[m] + c[m];
                sum += c[m];
            }
            t.fsrc[(size_t)mu * t.face_cap + k] = ((sum & 1) << 30) | (l2 >> 1);
        }
    // blocks in lexicographic order -> their place in the colour-major layout
    t.bord.assign(Nb, 0);
    for (int Bl = 0; Bl < Nb; ++Bl) {
        int r = Bl, bsum = 0;
        for (int m = 3; m >= 0; --m) {
            bsum += r % nb[m];
            r /= nb[m];
        }
        t.bord[Bl] = (bsum & 1) * (Nb / 2) + Bl / 2;
    }
    // block neighbours for the face exchange of the Schwarz sweeps
    t.fnb.assign((size_t)8 * Nb, 0);
    for (int Bl = 0; Bl < Nb; ++Bl) {
        int cb[4], r = Bl;
        for (int m = 3; m >= 0; --m) {
            cb[m] = r % nb[m];
            r /= nb[m];
        }
        for (int mu = 0; mu < 4; ++mu)
            for (int d = 0; d < 2; ++d) {
                int cc[4] = {cb[0], cb[1], cb[2], cb[3]};
                cc[mu] = (cc[mu] + (d == 0 ? -1 : 1) + nb[mu]) % nb[mu];
                int Rl = 0;
                for (int m = 0; m < 4; ++m) Rl = Rl * nb[m] + cc[m];
                // d = 0: the reader's forward face meets this block's first
                // time slice; d = 1: its backward face meets the last one
                const bool wrap = mu == 0 && (d == 0 ? cb[0] == 0 : cb[0] == nb[0] - 1);
                t.fnb[(size_t)t.bord[Bl] * 8 + 2 * mu + d] = t.bord[Rl] | ((wrap && bc_t == -1) ? (int)0x80000000u : 0);
            }
    }
}

}  // namespace dfl
