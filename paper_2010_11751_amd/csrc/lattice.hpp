// Compile-time description of the D3Q19 / D3Q27 stencils and of the Hermite
// basis used by the regularized collision models.
//
// The velocity set is generated, not tabulated: the first half holds the
// vectors of {-1,0,1}^3 (|c|^2 <= 2 for D3Q19) whose first nonzero component
// is -1, by number of nonzeros and then lexicographically; then the rest
// velocity; then the negatives of the first half. This puts c_0 = (-1,0,0)
// and c_10 = (1,0,0) on D3Q19, the pair of the worked example of Sec. 2.6.
// Weights: D3Q19 {1/3, 1/18, 1/36} by number of nonzeros; D3Q27 the tensor
// product of the 1-D weights {2/3, 1/6, 1/6} (as exact ratios n/216).
#pragma once

#include <cstdint>
#include <type_traits>

namespace lbm {

template <int Q>
struct Stencil {
    static_assert(Q == 19 || Q == 27, "D3Q19 or D3Q27");
    static constexpr int q = Q;
    static constexpr int half = (Q - 1) / 2;
    static constexpr int rest = half;
    int c[Q][3];
    double t[Q];
    int opp[Q];
};

template <int Q>
constexpr Stencil<Q> make_stencil()
{
    Stencil<Q> s{};
    constexpr int H = Stencil<Q>::half;
    int n = 0;
    for (int nnz = 1; nnz <= 3; ++nnz)
        for (int a = -1; a <= 1; ++a)
            for (int b = -1; b <= 1; ++b)
                for (int e = -1; e <= 1; ++e) {
                    const int cnt = (a != 0) + (b != 0) + (e != 0);
                    if (cnt != nnz || (Q == 19 && cnt == 3)) continue;
                    const int first = a != 0 ? a : (b != 0 ? b : e);
                    if (first != -1) continue;
                    s.c[n][0] = a;
                    s.c[n][1] = b;
                    s.c[n][2] = e;
                    ++n;
                }
    for (int k = 0; k < H; ++k)
        for (int d = 0; d < 3; ++d) s.c[k + H + 1][d] = -s.c[k][d];
    s.c[H][0] = s.c[H][1] = s.c[H][2] = 0;
    for (int k = 0; k < Q; ++k) {
        const int cnt = (s.c[k][0] != 0) + (s.c[k][1] != 0) + (s.c[k][2] != 0);
        if (Q == 19) {
            const int num = cnt == 0 ? 12 : cnt == 1 ? 2 : 1;
            s.t[k] = double(num) / 36.0;
        } else {
            int num = 1;
            for (int d = 0; d < 3; ++d) num *= s.c[k][d] == 0 ? 4 : 1;
            s.t[k] = double(num) / 216.0;
        }
        s.opp[k] = k == H ? H : (k < H ? k + H + 1 : k - H - 1);
    }
    return s;
}

template <int Q>
struct L {
    static constexpr Stencil<Q> s = make_stencil<Q>();
    static constexpr int q = Q;
    static constexpr int half = Stencil<Q>::half;
    static constexpr int rest = Stencil<Q>::rest;
    static constexpr int cx(int k) { return s.c[k][0]; }
    static constexpr int cy(int k) { return s.c[k][1]; }
    static constexpr int cz(int k) { return s.c[k][2]; }
    static constexpr int c(int k, int d) { return s.c[k][d]; }
    static constexpr double t(int k) { return s.t[k]; }
    static constexpr int opp(int k) { return s.opp[k]; }
};

// ---------------------------------------------------------------------------
// Hermite basis. A multi-index n = (n_x, n_y, n_z) in {0,1,2}^3 names the
// tensor-product polynomial H_n(c) = prod_a h_{n_a}(c_a) with h_0 = 1,
// h_1(c) = c, h_2(c) = c^2 - 1/3, of norm N_n = prod_a n_a! * (1/3)^|n|.
// Support set S of the recursive-regularized model: all 27 on D3Q27; on
// D3Q19 the 10 of order <= 2 and the six permutations of (2,1,0). The
// regularized model keeps only the orders <= 2.

struct MultiIndex {
    int n[3];
};

constexpr double hermite_1d(int n, int c) { return n == 0 ? 1.0 : n == 1 ? double(c) : double(c * c) - 1.0 / 3.0; }

constexpr int order(const MultiIndex& m) { return m.n[0] + m.n[1] + m.n[2]; }

constexpr double hermite_norm(const MultiIndex& m)
{
    double v = 1.0;
    for (int d = 0; d < 3; ++d) {
        if (m.n[d] >= 1) v *= 1.0 / 3.0;
        if (m.n[d] == 2) v *= 2.0 / 3.0;
    }
    return v;
}

template <int Q, bool RECURSIVE>
constexpr bool in_support(int a, int b, int e)
{
    const int ord = a + b + e;
    if (ord <= 2) return true;
    if (!RECURSIVE) return false;
    if (Q == 27) return true;
    const int twos = (a == 2) + (b == 2) + (e == 2);
    const int ones = (a == 1) + (b == 1) + (e == 1);
    return ord == 3 && twos == 1 && ones == 1;
}

template <int Q, bool RECURSIVE>
constexpr int support_size()
{
    int n = 0;
    for (int a = 0; a <= 2; ++a)
        for (int b = 0; b <= 2; ++b)
            for (int e = 0; e <= 2; ++e) n += in_support<Q, RECURSIVE>(a, b, e);
    return n;
}

template <int Q, bool RECURSIVE>
struct Support {
    static constexpr int size = support_size<Q, RECURSIVE>();
    MultiIndex m[size > 0 ? size : 1];
};

template <int Q, bool RECURSIVE>
constexpr Support<Q, RECURSIVE> make_support()
{
    Support<Q, RECURSIVE> s{};
    int n = 0;
    for (int ord = 0; ord <= 6; ++ord)
        for (int a = 0; a <= 2; ++a)
            for (int b = 0; b <= 2; ++b)
                for (int e = 0; e <= 2; ++e)
                    if (a + b + e == ord && in_support<Q, RECURSIVE>(a, b, e)) s.m[n++] = MultiIndex{{a, b, e}};
    return s;
}

template <int Q, bool RECURSIVE>
struct HS {
    static constexpr Support<Q, RECURSIVE> s = make_support<Q, RECURSIVE>();
    static constexpr int size = Support<Q, RECURSIVE>::size;
    static constexpr MultiIndex m(int j) { return s.m[j]; }
    // H_n(c_k) / N_n
    static constexpr double coef(int j, int k)
    {
        const MultiIndex mi = s.m[j];
        double h = 1.0;
        for (int d = 0; d < 3; ++d) h *= hermite_1d(mi.n[d], L<Q>::c(k, d));
        return h / hermite_norm(mi);
    }
};

// Compile-time loop: f(std::integral_constant<int, I>) for I in [B, E).
template <int B, int E, class F>
__host__ __device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

}  // namespace lbm
