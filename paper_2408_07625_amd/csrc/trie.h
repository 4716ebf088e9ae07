// Prefix trees of U and of the unique XY set, and their simultaneous walk
// (LoopOverTrie, Alg. 2C; tree construction, Alg. 3).
//
// A trie over sorted unique keys is kept in path-compressed form: a binary
// radix tree whose internal nodes are the branch points.  An internal node
// covers a contiguous range of the sorted keys that share every bit above the
// node's branch bit; its left child holds the keys with that bit 0, its right
// child those with the bit 1.  The tree is built in parallel, one thread per
// internal node, by the construction of T. Karras, "Maximizing parallelism in
// the construction of BVHs, octrees, and k-d trees" (HPG 2012).  Bits are
// visited from the most significant qubit (64 W - 1) down to qubit 0; the
// set of coupled pairs does not depend on the order in which qubits are
// visited.
//
// The walk pairs a node u of the U tree with a node v of the XY tree.  All
// keys below u agree on the bits above u's branch bit, and likewise for v, so
// between two branch points the condition x'_b = x_b ^ XY_b of the paper's
// level-by-level walk is checked for a whole run of bits at once with one
// masked XOR of x ^ key(u) ^ key(v).  At a branch bit b the walk follows,
// for x'_b in {0, 1}, the U child with bit x'_b and the XY child with bit
// x_b ^ x'_b, keeping the pair only if both exist.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace eloc {

struct TNode {
    int32_t left;    // >= 0 internal node, < 0 leaf ~index
    int32_t right;
    int32_t rep;     // a leaf inside the node's range
    int32_t bit;     // branch bit, 0 .. 64 W - 1
};

constexpr int32_t kNoNode = INT32_MIN;

// Common prefix length (from the most significant bit) of keys i and j of a
// sorted array K[n][W]; -1 if j is outside [0, n).
template <int W>
__host__ __device__ inline int trie_cpl(const uint64_t* K, int64_t n, int64_t i, int64_t j) {
    if (j < 0 || j >= n) return -1;
    for (int w = W - 1; w >= 0; --w) {
        const uint64_t d = K[i * W + w] ^ K[j * W + w];
        if (d) return (W - 1 - w) * 64 + __builtin_clzll(d);
    }
    return 64 * W;
}

// Internal node i (0 <= i < n - 1) of the radix tree over K[n][W]; node 0 is
// the root.
template <int W>
__host__ __device__ inline TNode trie_node(const uint64_t* K, int64_t n, int64_t i) {
    const int dir = (trie_cpl<W>(K, n, i, i + 1) - trie_cpl<W>(K, n, i, i - 1)) > 0 ? 1 : -1;
    const int dmin = trie_cpl<W>(K, n, i, i - dir);
    int64_t lmax = 2;
    while (trie_cpl<W>(K, n, i, i + lmax * dir) > dmin) lmax *= 2;
    int64_t l = 0;
    for (int64_t t = lmax / 2; t >= 1; t /= 2)
        if (trie_cpl<W>(K, n, i, i + (l + t) * dir) > dmin) l += t;
    const int64_t j = i + l * dir;
    const int dnode = trie_cpl<W>(K, n, i, j);
    int64_t s = 0;
    int64_t t = l;
    do {
        t = (t + 1) / 2;
        if (trie_cpl<W>(K, n, i, i + (s + t) * dir) > dnode) s += t;
    } while (t > 1);
    const int64_t gamma = i + s * dir + (dir < 0 ? -1 : 0);
    const int64_t lo = i < j ? i : j;
    const int64_t hi = i < j ? j : i;
    TNode nd;
    nd.left = (lo == gamma) ? ~static_cast<int32_t>(gamma) : static_cast<int32_t>(gamma);
    nd.right = (hi == gamma + 1) ? ~static_cast<int32_t>(gamma + 1) : static_cast<int32_t>(gamma + 1);
    nd.rep = static_cast<int32_t>(gamma);
    nd.bit = 64 * W - 1 - dnode;
    return nd;
}

template <int W>
__host__ __device__ inline int trie_bit(const uint64_t* k, int b) {
    return static_cast<int>((k[b >> 6] >> (b & 63)) & 1ull);
}

// true if (a ^ b ^ c) has no set bit in [lo, hi)
template <int W>
__host__ __device__ inline bool trie_agree(const uint64_t* a, const uint64_t* b, const uint64_t* c, int lo,
                                           int hi) {
    bool ok = true;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const int s = lo - 64 * w < 0 ? 0 : (lo - 64 * w > 64 ? 64 : lo - 64 * w);
        const int e = hi - 64 * w < 0 ? 0 : (hi - 64 * w > 64 ? 64 : hi - 64 * w);
        if (e > s) {
            const uint64_t up = e >= 64 ? ~0ull : ((1ull << e) - 1ull);
            const uint64_t dn = s >= 64 ? ~0ull : ((1ull << s) - 1ull);
            ok = ok && (((a[w] ^ b[w] ^ c[w]) & (up & ~dn)) == 0ull);
        }
    }
    return ok;
}

// One tree: sorted keys K[n][W], internal nodes N[n-1] with the key of each
// node's representative leaf beside them (nkeys[n-1][W], so that a node and
// its key are loaded together), root 0 (or leaf ~0 when n == 1).
struct TrieView {
    const uint64_t* keys;
    const TNode* nodes;
    const uint64_t* nkeys;
    int64_t n;
};

// Walk U x XY for the row key x and call on_hit(u_leaf, v_leaf) for every
// pair of leaves with x ^ key(u) == key(v).  Stack depth is bounded by the
// number of bits (each pushed entry sits at a strictly smaller branch bit).
template <int W, class OnHit>
__host__ __device__ inline void trie_walk(const uint64_t* x, const TrieView& U, const TrieView& V,
                                          OnHit&& on_hit) {
    if (U.n <= 0 || V.n <= 0) return;
    int32_t su[64 * W];
    int32_t sv[64 * W];
    int16_t sd[64 * W];
    int sp = 0;
    int32_t u = U.n > 1 ? 0 : ~0;
    int32_t v = V.n > 1 ? 0 : ~0;
    int d = 64 * W;
    for (;;) {
        bool next = false;
        const TNode nu = u >= 0 ? U.nodes[u] : TNode{0, 0, ~u, -1};
        const TNode nv = v >= 0 ? V.nodes[v] : TNode{0, 0, ~v, -1};
        const uint64_t* ku = u >= 0 ? U.nkeys + static_cast<int64_t>(u) * W : U.keys + static_cast<int64_t>(~u) * W;
        const uint64_t* kv = v >= 0 ? V.nkeys + static_cast<int64_t>(v) * W : V.keys + static_cast<int64_t>(~v) * W;
        const int b = nu.bit > nv.bit ? nu.bit : nv.bit;
        if (trie_agree<W>(x, ku, kv, b + 1, d)) {
            if (b < 0) {
                on_hit(nu.rep, nv.rep);
            } else {
                const int xb = trie_bit<W>(x, b);
                int32_t u0, u1, v0, v1;
                if (nu.bit == b) {
                    u0 = nu.left;
                    u1 = nu.right;
                } else {
                    const int ub = trie_bit<W>(ku, b);
                    u0 = ub ? kNoNode : u;
                    u1 = ub ? u : kNoNode;
                }
                if (nv.bit == b) {
                    v0 = nv.left;
                    v1 = nv.right;
                } else {
                    const int vb = trie_bit<W>(kv, b);
                    v0 = vb ? kNoNode : v;
                    v1 = vb ? v : kNoNode;
                }
                // x'_b = 0 pairs the U child 0 with the XY child x_b; x'_b = 1
                // the U child 1 with the XY child 1 - x_b.
                const int32_t a_u = u0, a_v = xb ? v1 : v0;
                const int32_t c_u = u1, c_v = xb ? v0 : v1;
                const bool a_ok = a_u != kNoNode && a_v != kNoNode;
                const bool c_ok = c_u != kNoNode && c_v != kNoNode;
                if (a_ok && c_ok) {
                    su[sp] = c_u;
                    sv[sp] = c_v;
                    sd[sp] = static_cast<int16_t>(b);
                    ++sp;
                }
                if (a_ok) {
                    u = a_u;
                    v = a_v;
                    d = b;
                    next = true;
                } else if (c_ok) {
                    u = c_u;
                    v = c_v;
                    d = b;
                    next = true;
                }
            }
        }
        if (next) continue;
        if (sp == 0) break;
        --sp;
        u = su[sp];
        v = sv[sp];
        d = sd[sp];
    }
}

}  // namespace eloc
