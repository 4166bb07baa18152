// Compile-time Tanner-graph block patterns of the supported quasi-cyclic codes.
//
// A quasi-cyclic matrix is a base_m x base_n array of L x L blocks, each zero
// or a circulant permutation P^a (P^a[r][(r + a) mod L] = 1).  The decoder
// kernels fix the block *pattern* (which blocks are nonzero) at compile time
// and take the circulant shifts at run time, so every loop over the Tanner
// graph unrolls into straight-line code with constant LDS offsets.
//
// Pattern of the lifted-product code LP(A, A*) with a 3 x 5 base A whose
// entries are all monomials (Section 2 uses such CSS pairs; the family is
// Panteleev and Kalachev's), Kronecker index (i, k) -> i * dim + k:
//   H_Z = [I_5 (x) A | A* (x) I_3]   H_X = [A (x) I_5 | I_3 (x) A*]
// Both are 15 x 34 blocks; every block row has 8 nonzero blocks (check
// degree 8), the first 25 block columns have 3 and the last 9 have 5.
#pragma once
#include <stdint.h>

#include <type_traits>
#include <utility>

namespace qldpc {

// Compile-time loop: f(std::integral_constant<int, I>{}) for I = B .. E-1.
template <int B, int E, class F>
__host__ __device__ __forceinline__ constexpr void static_for(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(std::forward<F>(f));
    }
}

constexpr int kMaxDv = 5;

struct PatternTables {
    int slot_bc[15][8];      // block column of slot j in block row R (increasing)
    int col_deg[34];         // nonzero blocks in block column C
    int col_R[34][kMaxDv];   // their block rows, increasing
    int col_j[34][kMaxDv];   // their slot index within that block row
    constexpr int ncols() const { return 34; }
};

// which = 0: H_Z side, 1: H_X side.
constexpr bool lp35_nonzero(int which, int R, int C) {
    constexpr int ma = 3, na = 5, off = na * na;
    if (which == 0) {
        // I_5 (x) A: rows (k, i) -> k*3 + i, cols (l, j) -> l*5 + j, k == l
        // A* (x) I_3: rows (c, b) -> c*3 + b, cols (e, d) -> 25 + e*3 + d, b == d
        if (C < off) return (R / ma) == (C / na);
        return (R % ma) == ((C - off) % ma);
    }
    // A (x) I_5: rows (i, k) -> i*5 + k, cols (j, l) -> j*5 + l, k == l
    // I_3 (x) A*: rows (b, c) -> b*5 + c, cols (d, e) -> 25 + d*3 + e, b == d
    if (C < off) return (R % na) == (C % na);
    return (R / na) == ((C - off) / ma);
}

constexpr PatternTables make_lp35(int which) {
    PatternTables t{};
    for (int R = 0; R < 15; ++R) {
        int j = 0;
        for (int C = 0; C < 34; ++C)
            if (lp35_nonzero(which, R, C)) t.slot_bc[R][j++] = C;
    }
    for (int C = 0; C < 34; ++C) {
        int d = 0;
        for (int R = 0; R < 15; ++R)
            for (int j = 0; j < 8; ++j)
                if (t.slot_bc[R][j] == C) {
                    t.col_R[C][d] = R;
                    t.col_j[C][d] = j;
                    ++d;
                }
        t.col_deg[C] = d;
    }
    return t;
}

struct ShapeLP35Z {
    static constexpr int MB = 15, NB = 34, DC = 8, SLOTS = MB * DC, WHICH = 0;
    static constexpr PatternTables T = make_lp35(0);
};
struct ShapeLP35X {
    static constexpr int MB = 15, NB = 34, DC = 8, SLOTS = MB * DC, WHICH = 1;
    static constexpr PatternTables T = make_lp35(1);
};

}  // namespace qldpc
