// Exercises the library's host-only argument checks and the sliced-ELL and
// padded row image builders on valid and malformed CSR inputs, for a build with the address
// and undefined-behaviour sanitizers (no HIP runtime call is made).  Prints
// "ok" and exits 0 when every check returned what it should.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <vector>

#include "internal.hpp"

using namespace oim;

static int fails = 0;
static void check(bool ok, const char* what) {
    if (!ok) {
        std::printf("FAIL %s\n", what);
        ++fails;
    }
}

struct Csr {
    int32_t n;
    std::vector<int64_t> rp;
    std::vector<int32_t> col;
    std::vector<float> J;
};

// symmetric random graph on n vertices, rows in column order
static Csr random_graph(int32_t n, uint32_t seed, int per_mille) {
    std::vector<std::vector<float>> a(n, std::vector<float>(n, 0.f));
    uint32_t s = seed;
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            s = s * 1664525u + 1013904223u;
            if ((int)((s >> 8) % 1000) < per_mille) a[i][j] = a[j][i] = ((s >> 4) & 1) ? 1.f : -0.5f;
        }
    Csr g{n, {0}, {}, {}};
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j)
            if (a[i][j] != 0.f) {
                g.col.push_back(j);
                g.J.push_back(a[i][j]);
            }
        g.rp.push_back((int64_t)g.col.size());
    }
    return g;
}

static int validate(const Csr& g) {
    return validate_csr(g.n, (int64_t)g.col.size(), g.rp.data(), g.col.data(), g.J.data());
}

int main() {
    for (int32_t n : {1, 3, 255, 256, 257, 700, 1500}) {
        Csr g = random_graph(n, 7u + n, n > 500 ? 8 : 60);
        check(validate(g) == OIM_OK, "valid graph accepted");
        SellImage img;
        build_sell(g.n, g.rp.data(), g.col.data(), g.J.data(), 1, nullptr, img);
        check(img.slices == (n + 255) / 256, "slices");
        // two instances: the lower and upper halves of a block-diagonal graph
        if (n >= 4) {
            Csr a = random_graph(n / 2, 3u, 80), b = random_graph(n - n / 2, 4u, 80);
            Csr bd{n, {0}, {}, {}};
            for (int i = 0; i < a.n; ++i) {
                for (int64_t e = a.rp[i]; e < a.rp[i + 1]; ++e) {
                    bd.col.push_back(a.col[e]);
                    bd.J.push_back(a.J[e]);
                }
                bd.rp.push_back((int64_t)bd.col.size());
            }
            for (int i = 0; i < b.n; ++i) {
                for (int64_t e = b.rp[i]; e < b.rp[i + 1]; ++e) {
                    bd.col.push_back(b.col[e] + a.n);
                    bd.J.push_back(b.J[e]);
                }
                bd.rp.push_back((int64_t)bd.col.size());
            }
            const int32_t off[3] = {0, a.n, n};
            check(validate(bd) == OIM_OK, "block-diagonal accepted");
            check(validate_blocks(n, bd.rp.data(), bd.col.data(), 2, off) == OIM_OK, "blocks ok");
            const int32_t bad_off[3] = {0, a.n - 1, n};
            if (a.n > 1 && bd.rp[a.n] > bd.rp[a.n - 1])
                check(validate_blocks(n, bd.rp.data(), bd.col.data(), 2, bad_off) != OIM_OK,
                      "coupled instances rejected");
            SellImage bimg;
            build_sell(n, bd.rp.data(), bd.col.data(), bd.J.data(), 2, off, bimg);
            check(bimg.inst.size() == 2 && bimg.order.size() == 2, "batch image");
        }
    }
    // the unit-weight image: same rows, offsets alone, padding at the zero
    // entry after the table and colours
    for (int32_t n : {5, 300, 900}) {
        Csr g = random_graph(n, 21u + n, 30);
        for (float& w : g.J) w = -1.f;
        SellImage img;
        build_sell(g.n, g.rp.data(), g.col.data(), g.J.data(), 1, nullptr, img, -1.f);
        check(img.entries_uw.size() == img.entries.size(), "unit-weight image size");
        const uint32_t zoff = (uint32_t)(36 * 64 * img.slices);
        size_t real = 0;
        for (uint32_t o : img.entries_uw) {
            check(o == zoff || o < (uint32_t)(32 * 64 * img.slices), "offset in the table or zero");
            real += o != zoff;
        }
        check(real == g.col.size(), "every stored entry once");
        SellImage plain;
        build_sell(g.n, g.rp.data(), g.col.data(), g.J.data(), 1, nullptr, plain, 0.f);
        check(plain.entries_uw.empty(), "no unit-weight image without a uniform weight");
        // row splits: (first entry with column > the row, row length)
        check(img.row_split.size() == (size_t)img.slices * 256, "row split size");
        for (int s = 0; s < img.slices; ++s)
            for (int j = 0; j < 4; ++j)
                for (int l = 0; l < 64; ++l) {
                    const int i = 4 * (s * 64 + l) + j;
                    const int2 sp = img.row_split[(s * 4 + j) * 64 + l];
                    if (i >= n) {
                        check(sp.x == 0 && sp.y == 0, "padding row split");
                        continue;
                    }
                    check(sp.y == (int)(g.rp[i + 1] - g.rp[i]) && sp.x <= sp.y, "row split length");
                    for (int k = 0; k < sp.y; ++k)
                        check((g.col[g.rp[i] + k] > i) == (k >= sp.x), "row split point");
                }
    }
    // the stepwise loop's padded row image: every row of every quad D
    // entries in CSR order, padding of weight 0 pointing at the row itself
    for (int32_t n : {1, 5, 64, 301}) {
        Csr g = random_graph(n, 31u + n, 40);
        check(ell_wanted(g.n, g.rp.data(), 1) && !ell_wanted(g.n, g.rp.data(), 0), "ell modes");
        EllImage ell;
        build_ell(g.n, g.rp.data(), g.col.data(), g.J.data(), ell);
        int64_t dmax = 0;
        for (int i = 0; i < n; ++i) dmax = std::max<int64_t>(dmax, g.rp[i + 1] - g.rp[i]);
        check(ell.D % 4 == 0 && ell.D >= 4 && ell.D >= dmax && ell.D < dmax + 4 + (dmax == 0 ? 4 : 0),
              "ell row length");
        const int np = (n + 3) / 4 * 4;
        check(ell.col.size() == (size_t)np * ell.D && ell.J.size() == ell.col.size(), "ell size");
        for (int i = 0; i < np; ++i)
            for (int e = 0; e < ell.D; ++e) {
                const size_t x = (size_t)(i / 4) * 4 * ell.D + (e / 4) * 16 + (i % 4) * 4 + e % 4;
                const int64_t len = i < n ? g.rp[i + 1] - g.rp[i] : 0;
                if (e < len) {
                    check(ell.col[x] == g.col[g.rp[i] + e] && ell.J[x] == g.J[g.rp[i] + e],
                          "ell entry");
                } else {
                    check(ell.J[x] == 0.f && ell.col[x] == std::min(i, n - 1), "ell padding");
                }
            }
    }
    {
        // similar rows take the image by default, a hub row does not
        Csr ring{8, {0}, {}, {}};
        for (int i = 0; i < 8; ++i) {
            ring.col.push_back((i + 7) % 8);
            ring.col.push_back((i + 1) % 8);
            ring.J.push_back(1.f);
            ring.J.push_back(1.f);
            ring.rp.push_back((int64_t)ring.col.size());
        }
        check(ell_wanted(ring.n, ring.rp.data(), 2), "ring takes the padded image");
        Csr star{64, {0}, {}, {}};
        for (int j = 1; j < 64; ++j) {
            star.col.push_back(j);
            star.J.push_back(1.f);
        }
        star.rp.push_back((int64_t)star.col.size());
        for (int i = 1; i < 64; ++i) {
            star.col.push_back(0);
            star.J.push_back(1.f);
            star.rp.push_back((int64_t)star.col.size());
        }
        check(!ell_wanted(star.n, star.rp.data(), 2), "star keeps the CSR");
    }
    // malformed inputs are rejected, never read out of bounds
    Csr g = random_graph(40, 11u, 150);
    {
        Csr h = g;
        h.col[0] = 40;  // out of range
        check(validate(h) != OIM_OK, "column out of range");
        h = g;
        h.col[0] = -1;
        check(validate(h) != OIM_OK, "negative column");
        h = g;
        h.J[0] = std::nanf("");
        check(validate(h) != OIM_OK, "NaN weight");
        h = g;
        h.J[0] *= 2.f;  // breaks symmetry
        check(validate(h) != OIM_OK, "asymmetric weight");
        h = g;
        h.rp[5] = h.rp[6] + 1;  // decreasing row pointers
        check(validate(h) != OIM_OK, "row pointers not monotone");
        h = g;
        h.rp[40] += 1;  // row_ptr[n] != nnz
        check(validate_csr(h.n, (int64_t)g.col.size(), h.rp.data(), h.col.data(), h.J.data()) !=
                  OIM_OK,
              "row_ptr[n] != nnz");
        // a self loop: row 0 gets an entry (0, 0)
        Csr s{g.n, {0}, {}, {}};
        s.col.push_back(0);
        s.J.push_back(1.f);
        for (int i = 0; i < g.n; ++i) {
            for (int64_t e = g.rp[i]; e < g.rp[i + 1]; ++e) {
                s.col.push_back(g.col[e]);
                s.J.push_back(g.J[e]);
            }
            s.rp.push_back((int64_t)s.col.size());
        }
        check(validate(s) != OIM_OK, "self loop");
    }
    std::vector<float> dense(9, 0.f);
    dense[1] = dense[3] = 1.f;
    check(validate_dense(3, dense.data()) == OIM_OK, "dense ok");
    dense[1] = 2.f;
    check(validate_dense(3, dense.data()) != OIM_OK, "dense asymmetric");
    if (fails) return 1;
    std::printf("ok\n");
    return 0;
}
