// Host build of the trie construction and walk (the same templates the GPU
// kernels instantiate), exercised by tests/test_trie_host.py against brute
// force on the CPU.
#include "trie.h"

#include <cstdint>
#include <vector>

using namespace eloc;

template <int W>
static int64_t run(const uint64_t* U, int64_t nU, const uint64_t* V, int64_t nV, const uint64_t* X, int64_t nX,
                   int64_t cap, int64_t* out_row, int64_t* out_u, int64_t* out_v, int32_t* nodes_out) {
    std::vector<TNode> un(nU > 1 ? nU - 1 : 1), vn(nV > 1 ? nV - 1 : 1);
    std::vector<uint64_t> uk(un.size() * W), vk(vn.size() * W);
    for (int64_t i = 0; i + 1 < nU; ++i) {
        un[i] = trie_node<W>(U, nU, i);
        for (int w = 0; w < W; ++w) uk[i * W + w] = U[un[i].rep * W + w];
    }
    for (int64_t i = 0; i + 1 < nV; ++i) {
        vn[i] = trie_node<W>(V, nV, i);
        for (int w = 0; w < W; ++w) vk[i * W + w] = V[vn[i].rep * W + w];
    }
    for (int64_t i = 0; i + 1 < nU; ++i) {
        nodes_out[4 * i] = un[i].left;
        nodes_out[4 * i + 1] = un[i].right;
        nodes_out[4 * i + 2] = un[i].rep;
        nodes_out[4 * i + 3] = un[i].bit;
    }
    TrieView tu{U, un.data(), uk.data(), nU}, tv{V, vn.data(), vk.data(), nV};
    int64_t count = 0;
    for (int64_t r = 0; r < nX; ++r) {
        trie_walk<W>(X + r * W, tu, tv, [&](int32_t a, int32_t b) {
            if (count < cap) {
                out_row[count] = r;
                out_u[count] = a;
                out_v[count] = b;
            }
            ++count;
        });
    }
    return count;
}

extern "C" int64_t trie_pairs_host(int W, const uint64_t* U, int64_t nU, const uint64_t* V, int64_t nV,
                                   const uint64_t* X, int64_t nX, int64_t cap, int64_t* out_row, int64_t* out_u,
                                   int64_t* out_v, int32_t* nodes_out) {
    if (W == 1) return run<1>(U, nU, V, nV, X, nX, cap, out_row, out_u, out_v, nodes_out);
    return run<2>(U, nU, V, nV, X, nX, cap, out_row, out_u, out_v, nodes_out);
}
