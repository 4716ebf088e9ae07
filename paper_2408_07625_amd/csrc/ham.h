// Host side of the Hamiltonian ingest (shared by the single-problem context
// and the batched launch): grouping of the terms by their XY mask in
// first-appearance order, the CSR of term runs with the even-|Y| / odd-|Y|
// split, the signed coefficients, the linear hash of every XY mask and the
// XY masks sorted for the prefix trees.
#pragma once

#include "internal.h"

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

namespace eloc {

// Growable open-addressing map keyed by W mask words.
struct XYMap {
    int W;
    std::vector<uint64_t> keys;
    std::vector<int64_t> vals;   // -1 = empty
    size_t count = 0;
    explicit XYMap(int w) : W(w) { resize(1024); }
    static uint64_t mix(uint64_t h) {
        h ^= h >> 33;
        h *= 0xff51afd7ed558ccdull;
        h ^= h >> 33;
        h *= 0xc4ceb9fe1a85ec53ull;
        return h ^ (h >> 33);
    }
    uint64_t hash(const uint64_t* k) const {
        uint64_t h = mix(k[0]);
        if (W == 2) h = mix(h ^ (k[1] + 0x9E3779B97F4A7C15ull));
        return h;
    }
    void resize(size_t cap) {
        std::vector<uint64_t> ok;
        std::vector<int64_t> ov;
        ok.swap(keys);
        ov.swap(vals);
        keys.assign(cap * W, 0);
        vals.assign(cap, -1);
        count = 0;
        for (size_t s = 0; s < ov.size(); ++s)
            if (ov[s] >= 0) insert(&ok[s * W], ov[s]);
    }
    // returns the existing value or inserts v
    int64_t find_or_insert(const uint64_t* k, int64_t v) {
        if (2 * (count + 1) > vals.size()) resize(vals.size() * 2);
        return insert(k, v);
    }
    int64_t insert(const uint64_t* k, int64_t v) {
        const size_t mask = vals.size() - 1;
        size_t s = hash(k) & mask;
        for (;;) {
            if (vals[s] < 0) {
                for (int w = 0; w < W; ++w) keys[s * W + w] = k[w];
                vals[s] = v;
                ++count;
                return v;
            }
            bool eq = true;
            for (int w = 0; w < W; ++w) eq = eq && keys[s * W + w] == k[w];
            if (eq) return vals[s];
            s = (s + 1) & mask;
        }
    }
};

template <int W>
struct HostHam {
    int64_t n_terms = 0;
    int64_t G = 0;
    int maxpop = 0;
    int diag = -1;
    int64_t maxpart = 0;             // longest real or imaginary part of a group's run
    std::vector<GroupRec<W>> groups;
    std::vector<TermRec<W>> terms;
    std::vector<TermRecF<W>> terms_f;
    std::vector<int32_t> term_src;   // caller index of every stored term
    std::vector<uint8_t> term_ny;    // its |Y| mod 4
    std::vector<uint64_t> ghash;     // lin(XY_g)
    std::vector<uint64_t> gkeys;     // XY_g [G][W]
    std::vector<int32_t> order;      // group ids sorted by XY (top word first)
    std::vector<uint64_t> xsorted;   // XY masks in that order [G][W]
};

// xy / yz: [n_terms][W]; R: the 64 W words of the linear hash.  Returns an
// empty string on success, else the reason.
template <int W>
std::string build_host_ham(const uint64_t* R, int64_t n_terms, const double* coeff, const uint64_t* xy,
                           const uint64_t* yz, HostHam<W>& out) {
    XYMap map(W);
    std::vector<int64_t> gid(static_cast<size_t>(n_terms));
    std::vector<int64_t> first;
    for (int64_t l = 0; l < n_terms; ++l) {
        const int64_t g = map.find_or_insert(xy + l * W, static_cast<int64_t>(first.size()));
        if (g == static_cast<int64_t>(first.size())) first.push_back(l);
        gid[static_cast<size_t>(l)] = g;
    }
    const int64_t G = static_cast<int64_t>(first.size());
    if (n_terms >= (int64_t(1) << 31) || G >= (int64_t(1) << 25))
        return "Hamiltonian too large (terms < 2^31, unique XY < 2^25)";
    // |Y| parity of each term: even terms form the real part of a group's
    // run, odd terms the imaginary part; i^|Y| = (-1)^floor(|Y|/2) i^(|Y| mod 2)
    std::vector<int> ny(static_cast<size_t>(n_terms));
    for (int64_t l = 0; l < n_terms; ++l) {
        int k = 0;
        for (int w = 0; w < W; ++w) k += __builtin_popcountll(xy[l * W + w] & yz[l * W + w]);
        ny[static_cast<size_t>(l)] = k;
    }
    std::vector<int64_t> n_even(static_cast<size_t>(G), 0), n_all(static_cast<size_t>(G), 0);
    for (int64_t l = 0; l < n_terms; ++l) {
        ++n_all[static_cast<size_t>(gid[l])];
        if ((ny[static_cast<size_t>(l)] & 1) == 0) ++n_even[static_cast<size_t>(gid[l])];
    }
    std::vector<int64_t> begin(static_cast<size_t>(G + 1), 0);
    for (int64_t g = 0; g < G; ++g) begin[g + 1] = begin[g] + n_all[static_cast<size_t>(g)];
    std::vector<int64_t> pos_even(begin.begin(), begin.end() - 1), pos_odd(static_cast<size_t>(G));
    for (int64_t g = 0; g < G; ++g) pos_odd[static_cast<size_t>(g)] = begin[g] + n_even[static_cast<size_t>(g)];
    out.n_terms = n_terms;
    out.G = G;
    out.terms.resize(static_cast<size_t>(n_terms));
    out.terms_f.resize(static_cast<size_t>(n_terms));
    out.term_src.resize(static_cast<size_t>(n_terms));
    out.term_ny.resize(static_cast<size_t>(n_terms));
    for (int64_t l = 0; l < n_terms; ++l) {   // caller order kept inside each part
        const size_t g = static_cast<size_t>(gid[l]);
        const int k = ny[static_cast<size_t>(l)];
        const int64_t p = (k & 1) ? pos_odd[g]++ : pos_even[g]++;
        const double h = ((k >> 1) & 1) ? -coeff[l] : coeff[l];
        TermRec<W> t;
        TermRecF<W> tf;
        for (int w = 0; w < W; ++w) {
            t.yz[w] = yz[l * W + w];
            tf.yz[w] = yz[l * W + w];
        }
        t.h = h;
        tf.h_hi = static_cast<float>(h);
        tf.h_lo = static_cast<float>(h - static_cast<double>(tf.h_hi));
        out.terms[static_cast<size_t>(p)] = t;
        out.terms_f[static_cast<size_t>(p)] = tf;
        out.term_src[static_cast<size_t>(p)] = static_cast<int32_t>(l);
        out.term_ny[static_cast<size_t>(p)] = static_cast<uint8_t>(k & 3);
    }
    out.groups.resize(static_cast<size_t>(G));
    out.ghash.resize(static_cast<size_t>(G));
    out.gkeys.resize(static_cast<size_t>(G * W));
    out.maxpop = 0;
    out.maxpart = 0;
    out.diag = -1;
    for (int64_t g = 0; g < G; ++g) {
        GroupRec<W> r;
        const uint64_t* m = xy + first[static_cast<size_t>(g)] * W;
        uint64_t h = 0;
        int pc = 0;
        for (int w = 0; w < W; ++w) {
            r.xy[w] = m[w];
            out.gkeys[static_cast<size_t>(g * W + w)] = m[w];
            pc += __builtin_popcountll(m[w]);
            for (uint64_t v = m[w]; v; v &= v - 1) h ^= R[64 * w + __builtin_ctzll(v)];
        }
        r.begin = static_cast<int32_t>(begin[static_cast<size_t>(g)]);
        r.mid = static_cast<int32_t>(begin[static_cast<size_t>(g)] + n_even[static_cast<size_t>(g)]);
        r.end = static_cast<int32_t>(begin[static_cast<size_t>(g + 1)]);
        r.pad = 0;
        out.groups[static_cast<size_t>(g)] = r;
        out.ghash[static_cast<size_t>(g)] = h;
        out.maxpop = std::max(out.maxpop, pc);
        out.maxpart = std::max<int64_t>(out.maxpart, std::max(r.mid - r.begin, r.end - r.mid));
        if (pc == 0) out.diag = static_cast<int>(g);
    }
    // masks sorted ascending (top word first) for the XY prefix trees
    out.order.resize(static_cast<size_t>(G));
    for (int64_t g = 0; g < G; ++g) out.order[static_cast<size_t>(g)] = static_cast<int32_t>(g);
    const std::vector<uint64_t>& gk = out.gkeys;
    std::sort(out.order.begin(), out.order.end(), [&](int32_t a, int32_t b) {
        for (int w = W - 1; w >= 0; --w) {
            const uint64_t ka = gk[static_cast<size_t>(a) * W + w], kb = gk[static_cast<size_t>(b) * W + w];
            if (ka != kb) return ka < kb;
        }
        return false;
    });
    out.xsorted.resize(static_cast<size_t>(G * W));
    for (int64_t i = 0; i < G; ++i)
        for (int w = 0; w < W; ++w)
            out.xsorted[static_cast<size_t>(i * W + w)] =
                gk[static_cast<size_t>(out.order[static_cast<size_t>(i)]) * W + w];
    return std::string();
}

}  // namespace eloc
