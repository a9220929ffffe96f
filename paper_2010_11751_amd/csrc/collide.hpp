// Collision models on one cell, fully unrolled over the stencil (the
// "unrolled" code style of Sec. 2.6: no multiplications by zero velocity
// components, terms of opposite populations shared through Eq. symmetry_Ek).
//
// Populations arrive either as f (FP64 storage) or shifted as g = f - t_k
// (FP32/FP16 storage). The arithmetic is written on the deviation so that it
// never forms 1 + small: with base = sum_k g_k (= rho - 1 when shifted, rho
// otherwise), every equilibrium is E_k - shift*t_k = t_k (base + rho*X_k).
// Results are returned in the same representation, in place.
#pragma once

#include "lattice.hpp"
#include "moments.hpp"

namespace lbm {

enum Model { BGK = 0, TRT = 1, REG = 2, RR = 3, NW4 = 4, RM = 5, HM = 6, CM = 7, CHM = 8, CUM = 9 };

template <class R>
struct Relax {
    R omega;    // shear relaxation omega_nu (TRT: omega_plus)
    R omega_m;  // TRT antisymmetric rate omega_minus
    R omega_b;  // bulk relaxation omega_nu_b (REG, RR, moment-space models)
    R omega3;   // third-order moments (moment-space models)
    R omega4;   // fourth and higher orders (moment-space models)
};

template <int Q, class R>
struct CellMoments {
    R s[L<Q>::half];  // g_k + g_kbar for k < half
    R d[L<Q>::half];  // g_k - g_kbar for k < half
    R base, rho, j[3], u[3];
};

template <int Q, bool SHIFT, class R>
__device__ __forceinline__ void cell_moments(const R (&g)[Q], CellMoments<Q, R>& m)
{
    using S = L<Q>;
    static_for<0, S::half>([&](auto K) {
        constexpr int k = K;
        m.s[k] = g[k] + g[S::opp(k)];
        m.d[k] = g[k] - g[S::opp(k)];
    });
    R rs = g[S::rest];
    R j[3] = {R(0), R(0), R(0)};
    static_for<0, S::half>([&](auto K) {
        constexpr int k = K;
        rs += m.s[k];
        static_for<0, 3>([&](auto D) {
            constexpr int a = D;
            if constexpr (S::c(k, a) == 1) j[a] += m.d[k];
            else if constexpr (S::c(k, a) == -1) j[a] -= m.d[k];
        });
    });
    m.base = rs;
    m.rho = SHIFT ? R(1) + rs : rs;
    const R inv = R(1) / m.rho;
    static_for<0, 3>([&](auto D) {
        m.j[D] = j[D];
        m.u[D] = j[D] * inv;
    });
}

// Second-order weighted equilibrium (BGK-W2, Sec. 2.6) split into the part
// even in c_k and the part odd in c_k: E_k = sym_k + anti_k, E_kbar = sym_k -
// anti_k, which is Eq. symmetry_Ek with anti_k = 3 t_k c_k.(rho u). The odd
// part is formed from the momentum j = rho u itself, so that the rounding of
// rho = 1 + base in FP32 never enters the linear term.
template <int Q, class R>
struct Eq2 {
    R sym[L<Q>::half];
    R anti[L<Q>::half];
    R rest;
};

template <int Q, class R>
__device__ __forceinline__ void equilibrium2(R base, R rho, const R (&j)[3], const R (&u)[3], Eq2<Q, R>& e)
{
    using S = L<Q>;
    const R usq15 = R(1.5) * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    e.rest = R(S::t(S::rest)) * (base - rho * usq15);
    static_for<0, S::half>([&](auto K) {
        constexpr int k = K;
        R cu = R(0), cj = R(0);
        static_for<0, 3>([&](auto D) {
            constexpr int a = D;
            if constexpr (S::c(k, a) == 1) {
                cu += u[a];
                cj += j[a];
            } else if constexpr (S::c(k, a) == -1) {
                cu -= u[a];
                cj -= j[a];
            }
        });
        const R tk = R(S::t(k));
        e.sym[k] = tk * (base + rho * (R(4.5) * cu * cu - usq15));
        e.anti[k] = (tk * R(3)) * cj;
    });
}

// Hermite coefficient A_n of the regularized models for the compile-time
// multi-index J of the support set: A_0 = base, A_a = j_a (= rho u_a), and for
// |n| >= 2, A_n = rho u^n + a1_n where a1_n is the relaxed non-equilibrium
// coefficient: Pi*_ab at order two and, beyond, the pair-sum recursion
// a1_{a1..am} = sum_{l<j} (prod_{r != l,j} u_{ar}) Pi*_{al aj}.
struct IndexList {
    int idx[6];
    int len;
};

constexpr IndexList index_list(MultiIndex m)
{
    IndexList l{};
    l.len = 0;
    for (int d = 0; d < 3; ++d)
        for (int r = 0; r < m.n[d]; ++r) l.idx[l.len++] = d;
    return l;
}

template <int Q, bool REC, int J, class R>
__device__ __forceinline__ R hermite_coefficient(R base, R rho, const R (&j)[3], const R (&u)[3], const R (&P)[3][3])
{
    constexpr MultiIndex mi = HS<Q, REC>::m(J);
    constexpr IndexList il = index_list(mi);
    if constexpr (il.len == 0) {
        return base;
    } else if constexpr (il.len == 1) {
        return j[il.idx[0]];
    } else {
        R un = j[il.idx[0]];
        static_for<1, il.len>([&](auto Rr) { un *= u[il.idx[Rr]]; });
        {
            R a1 = R(0);
            static_for<0, il.len>([&](auto Lc) {
                constexpr int l = Lc;
                static_for<l + 1, il.len>([&](auto Jc) {
                    constexpr int jj = Jc;
                    R prod = P[il.idx[l]][il.idx[jj]];
                    static_for<0, il.len>([&](auto Rr) {
                        constexpr int r = Rr;
                        if constexpr (r != l && r != jj) prod *= u[il.idx[r]];
                    });
                    a1 += prod;
                });
            });
            return un + a1;
        }
    }
}

// Populations from Hermite coefficients: f_k = t_k sum_{n in S} H_n(c_k)
// A_n / N_n, evaluated as even and odd parts in c so that a pair (k, kbar)
// costs one evaluation.
template <int Q, bool REC, class R>
__device__ __forceinline__ void from_hermite(const R (&A)[HS<Q, REC>::size], R (&g)[Q])
{
    using S = L<Q>;
    using H = HS<Q, REC>;
    static_for<0, S::half + 1>([&](auto K) {
        constexpr int k = K;
        R ev = R(0), od = R(0);
        static_for<0, H::size>([&](auto Jc) {
            constexpr int j = Jc;
            constexpr double cf = H::coef(j, k);
            if constexpr (cf != 0.0) {
                if constexpr (order(H::m(j)) % 2 == 0) ev += R(cf) * A[j];
                else od += R(cf) * A[j];
            }
        });
        const R tk = R(S::t(k));
        if constexpr (k == S::rest) {
            g[k] = tk * ev;
        } else {
            g[k] = tk * (ev + od);
            g[S::opp(k)] = tk * (ev - od);
        }
    });
}

// Exact conservation of mass and momentum in FP32 arithmetic. Every model
// conserves rho and j exactly in real numbers, but with weights rounded to
// FP32 (3 t_k is 1/6 and 1/12 only up to a relative 3e-8) the collision
// scales j by the same 1 + O(1e-8) factor in every cell at every step, a drift
// that accumulates linearly. Returning the (tiny) mass and momentum residuals
// to the rest population and to the three axis pairs removes it; in exact
// arithmetic this changes nothing.
template <int Q, class R>
__device__ __forceinline__ void conserve(R (&g)[Q], R base, const R (&j)[3])
{
    using S = L<Q>;
    static_assert(S::c(0, 0) == -1 && S::c(1, 1) == -1 && S::c(2, 2) == -1, "k = 0, 1, 2 are -e_x, -e_y, -e_z");
    R mo = g[S::rest];
    R jo[3] = {R(0), R(0), R(0)};
    static_for<0, S::half>([&](auto K) {
        constexpr int k = K;
        mo += g[k] + g[S::opp(k)];
        const R dk = g[k] - g[S::opp(k)];
        static_for<0, 3>([&](auto D) {
            constexpr int a = D;
            if constexpr (S::c(k, a) == 1) jo[a] += dk;
            else if constexpr (S::c(k, a) == -1) jo[a] -= dk;
        });
    });
    g[S::rest] += base - mo;
    static_for<0, 3>([&](auto D) {
        constexpr int a = D;
        const R d = R(0.5) * (j[a] - jo[a]);
        g[S::opp(a)] += d;
        g[a] -= d;
    });
}

template <int Q, int MODEL, bool SHIFT, class R>
__device__ __forceinline__ void collide(R (&g)[Q], const Relax<R>& p)
{
    using S = L<Q>;
    CellMoments<Q, R> m;
    cell_moments<Q, SHIFT>(g, m);

    if constexpr (MODEL >= NW4) {
        constexpr int FAM = (MODEL == NW4 || MODEL == RM) ? FAM_RAW
                          : MODEL == HM ? FAM_HERMITE : MODEL == CHM ? FAM_CHERMITE : FAM_CENTRAL;
        MomentRates<R> r;
        if constexpr (MODEL == NW4) {
            // BGK with the NW4 equilibrium: every moment relaxes at omega.
            r = MomentRates<R>{p.omega, p.omega, R(0), p.omega, p.omega};
        } else {
            const R wm = (p.omega_b - p.omega) * R(1.0 / 3.0);
            r = MomentRates<R>{p.omega, wm + p.omega, wm, p.omega3, p.omega4};
        }
        collide_moment_space<Q, FAM, MODEL == CUM>(g, m.s, m.d, m.base, m.rho, m.u, r);
    } else if constexpr (MODEL == BGK || MODEL == TRT) {
        Eq2<Q, R> e;
        equilibrium2<Q>(m.base, m.rho, m.j, m.u, e);
        const R w = p.omega;
        g[S::rest] = g[S::rest] + w * (e.rest - g[S::rest]);
        if constexpr (MODEL == BGK) {
            static_for<0, S::half>([&](auto K) {
                constexpr int k = K, kb = S::opp(k);
                g[k] = g[k] + w * (e.sym[k] + e.anti[k] - g[k]);
                g[kb] = g[kb] + w * (e.sym[k] - e.anti[k] - g[kb]);
            });
        } else {
            const R wm = p.omega_m;
            static_for<0, S::half>([&](auto K) {
                constexpr int k = K, kb = S::opp(k);
                const R a = w * (R(0.5) * m.s[k] - e.sym[k]);
                const R b = wm * (R(0.5) * m.d[k] - e.anti[k]);
                g[k] = g[k] - a - b;
                g[kb] = g[kb] - a + b;
            });
        }
    } else {
        constexpr bool REC = MODEL == RR;
        using H = HS<Q, REC>;
        // Non-equilibrium stress Pi_ab = sum_k c_a c_b g_k - rho u_a u_b - base delta_ab/3
        // (second moments are even in c, so they only need the pair sums s_k).
        R P[3][3];
        static_for<0, 3>([&](auto A_) {
            constexpr int a = A_;
            static_for<a, 3>([&](auto B_) {
                constexpr int b = B_;
                R acc = R(0);
                static_for<0, S::half>([&](auto K) {
                    constexpr int k = K;
                    constexpr int cc = S::c(k, a) * S::c(k, b);
                    if constexpr (cc == 1) acc += m.s[k];
                    else if constexpr (cc == -1) acc -= m.s[k];
                });
                acc -= m.j[a] * m.u[b];
                if constexpr (a == b) acc -= m.base * R(1.0 / 3.0);
                P[a][b] = acc;
            });
        });
        // Relaxation with the bulk knob (Eq. bulk, read with M - M_eq): the
        // deviator relaxes with omega_nu, the trace with omega_nu_b.
        const R am = R(1) - p.omega;
        const R tr3 = (P[0][0] + P[1][1] + P[2][2]) * R(1.0 / 3.0);
        const R bt = (p.omega - p.omega_b) * tr3;
        static_for<0, 3>([&](auto A_) {
            constexpr int a = A_;
            static_for<a, 3>([&](auto B_) {
                constexpr int b = B_;
                P[a][b] = a == b ? am * P[a][b] + bt : am * P[a][b];
                P[b][a] = P[a][b];
            });
        });
        R A[H::size];
        static_for<0, H::size>([&](auto Jc) {
            constexpr int j = Jc;
            A[j] = hermite_coefficient<Q, REC, j>(m.base, m.rho, m.j, m.u, P);
        });
        from_hermite<Q, REC>(A, g);
    }
    if constexpr (SHIFT) conserve<Q>(g, m.base, m.j);
}

// Equilibrium of the model at (rho, u) in the storage representation
// (E^S of the support set for RR, the NW4 equilibrium for the moment-space
// models, BGK-W2 otherwise).
template <int Q, int MODEL, bool SHIFT, class R>
__device__ __forceinline__ void equilibrium(R rho, const R (&u)[3], R (&g)[Q])
{
    using S = L<Q>;
    const R base = SHIFT ? rho - R(1) : rho;
    const R j[3] = {rho * u[0], rho * u[1], rho * u[2]};
    if constexpr (MODEL >= NW4) {
        equilibrium_nw4<Q>(base, rho, u, g);
    } else if constexpr (MODEL == RR) {
        using H = HS<Q, true>;
        R P[3][3] = {{R(0), R(0), R(0)}, {R(0), R(0), R(0)}, {R(0), R(0), R(0)}};
        R A[H::size];
        static_for<0, H::size>([&](auto Jc) {
            constexpr int jj = Jc;
            A[jj] = hermite_coefficient<Q, true, jj>(base, rho, j, u, P);
        });
        from_hermite<Q, true>(A, g);
    } else {
        Eq2<Q, R> e;
        equilibrium2<Q>(base, rho, j, u, e);
        g[S::rest] = e.rest;
        static_for<0, S::half>([&](auto K) {
            constexpr int k = K;
            g[k] = e.sym[k] + e.anti[k];
            g[S::opp(k)] = e.sym[k] - e.anti[k];
        });
    }
}

}  // namespace lbm
