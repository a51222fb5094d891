// Compile-time program of the inner walk, shared by the host planner and the
// device kernels.
//
// The paper's swap sequence Upsilon(K) (Sec. 3 recursion, with the "+1" shift
// of the text and of the Sec. 5 recurrence):
//     Upsilon(2) = [1],  Upsilon(K) = Upsilon(K-1) : [K-1, ..., 1] : [i+1 | i in Upsilon(K-1)].
// Here indices are 0-based: swap j exchanges positions j and j+1.
//
// A walk emits, after each swap at j, the families "first j+1 variables ->
// every later variable": a swap changes only that one prefix set, and the
// sequence makes every prefix set new exactly once.  Run backwards (swaps in
// reverse order, starting from the forward walk's final ordering) the same
// orderings are visited in reverse and again every subset appears exactly once;
// the kernels alternate forward and backward walks so that the inner block's
// ordering only ever takes two values, both known at compile time.
#pragma once

#include <cstdint>

namespace gs {

constexpr int ups_len(int k) { return k <= 1 ? 0 : (1 << k) - k - 1; }

template <int K>
struct InnerProgram {
    static constexpr int N = ups_len(K);
    static constexpr int NA = N > 0 ? N : 1;
    int j_f[NA];      // forward swap positions (Upsilon(K), 0-based)
    int piv_f[NA];    // variable at position j+1 before the forward swap
    int mov_f[NA];    // variable at position j before it (it moves to j+1)
    int mask_f[NA];   // prefix set (bitmask of inner labels) created by the swap
    int j_r[NA];      // backward walk: Upsilon(K) reversed
    int piv_r[NA];
    int mov_r[NA];
    int mask_r[NA];
    int init_f[K + 1];  // prefix sets of the forward start ordering (identity)
    int init_r[K + 1];  // prefix sets of the backward start ordering
    int order_f[K];     // forward start ordering (identity)
    int order_r[K];     // backward start ordering = forward final ordering
};

template <int K>
constexpr InnerProgram<K> make_inner_program() {
    InnerProgram<K> p{};
    constexpr int N = InnerProgram<K>::N;
    int seq[InnerProgram<K>::NA] = {};
    int len = 0;
    if (K >= 2) seq[len++] = 0;
    for (int kk = 3; kk <= K; ++kk) {
        const int old = len;
        for (int t = kk - 2; t >= 0; --t) seq[len++] = t;
        for (int t = 0; t < old; ++t) seq[len++] = seq[t] + 1;
    }
    int ord[K] = {};
    for (int i = 0; i < K; ++i) {
        ord[i] = i;
        p.order_f[i] = i;
    }
    for (int pl = 0; pl <= K; ++pl) {
        int mk = 0;
        for (int i = 0; i < pl; ++i) mk |= 1 << ord[i];
        p.init_f[pl] = mk;
    }
    for (int t = 0; t < N; ++t) {
        const int j = seq[t];
        p.j_f[t] = j;
        p.piv_f[t] = ord[j + 1];
        p.mov_f[t] = ord[j];
        const int tmp = ord[j];
        ord[j] = ord[j + 1];
        ord[j + 1] = tmp;
        int mk = 0;
        for (int i = 0; i <= j; ++i) mk |= 1 << ord[i];
        p.mask_f[t] = mk;
    }
    for (int i = 0; i < K; ++i) p.order_r[i] = ord[i];
    for (int pl = 0; pl <= K; ++pl) {
        int mk = 0;
        for (int i = 0; i < pl; ++i) mk |= 1 << ord[i];
        p.init_r[pl] = mk;
    }
    for (int t = 0; t < N; ++t) {
        const int j = seq[N - 1 - t];
        p.j_r[t] = j;
        p.piv_r[t] = ord[j + 1];
        p.mov_r[t] = ord[j];
        const int tmp = ord[j];
        ord[j] = ord[j + 1];
        ord[j + 1] = tmp;
        int mk = 0;
        for (int i = 0; i <= j; ++i) mk |= 1 << ord[i];
        p.mask_r[t] = mk;
    }
    return p;
}

template <int K>
inline constexpr InnerProgram<K> kInner = make_inner_program<K>();

constexpr int popcount_c(int x) {
    int c = 0;
    while (x) {
        c += x & 1;
        x >>= 1;
    }
    return c;
}

// Largest inner block compiled into the kernels, and largest middle block.
constexpr int KS_MAX = 6;
constexpr int Q_MAX = 16;

// Per-sub-walk program word layout (two 32-bit words per sub-walk t):
//   w0: bits 0..15  set of middle variables in front of the inner block
//                   (bit p = middle variable with label ks + p)
//       bits 16..20 z = number of middle variables in front, after the transition
//       bits 21..25 lane (= label) of the middle variable that the middle swap moves
//                   from position p to p+1 (used by the adjoint to recover c, s)
//   w1: bit 0       a transition precedes this sub-walk (t > 0)
//       bit 1       the transition starts with a swap of two middle variables
//       bits 2..6   that swap's position p (middle positions p and p+1)
//       bits 8..12  lane (= label) of the pivot column of that swap
//       bit 13      a middle variable crosses the inner block leftwards (z -> z+1);
//                   otherwise the front middle variable crosses rightwards (z -> z-1)
//       bits 16..20 lane (= label) of the crossing middle variable
//       bits 24..28 z before the transition
struct SubWord {
    static constexpr uint32_t kHasTransition = 1u;
    static constexpr uint32_t kHasMid = 2u;
    static constexpr uint32_t kCrossLeft = 1u << 13;
};

}  // namespace gs
