// Moment-space collision models (Sec. 2.2, Sec. 2.6) in the non-weighted
// formulation: BGK with the fourth-order non-weighted equilibrium (NW4) and
// multi-relaxation-time models in raw (RM), Hermite (HM), central (CM),
// central Hermite (CHM) moments and in cumulants (K).
//
// Basis. A multi-index n in {0,1,2}^3 names the moment of c_x^nx c_y^ny c_z^nz.
// The basis holds those n whose monomial does not vanish on every velocity:
// all 27 on D3Q27, the 19 with at most two nonzero entries on D3Q19 (it has
// no velocity with three nonzero components). Q populations and their Q
// basis moments determine each other. The inverse is a product over the axes
// of the 1-D inverse of the three moments (1, c, c^2) on the three velocities
// (-1, 0, 1):  f(-1) = (M2 - M1)/2,  f(0) = M0 - M2,  f(+1) = (M2 + M1)/2.
// On D3Q19 the same product restricted to the basis is the inverse, because
// the dropped moments are identically zero there.
//
// Deviation form. The models relax X_n towards X_n^eq, so only the change
// X*_n - X_n has to travel back to populations: f_out = f + rho * sum_n
// Minv[k][n] (M*_n - M_n). Every quantity on the way is a small deviation
// (moments are normalised by rho and measured from the moments W_n of the
// lattice weights), so the shifted FP32/FP16 storage never forms 1 + small
// and the FP64 path is the same code.
#pragma once

#include "lattice.hpp"

namespace lbm {

template <int Q>
struct MomentBasis {
    MultiIndex m[Q];
};

template <int Q>
constexpr MomentBasis<Q> make_moment_basis()
{
    MomentBasis<Q> b{};
    int n = 0;
    for (int ord = 0; ord <= 6; ++ord)
        for (int x = 0; x <= 2; ++x)
            for (int y = 0; y <= 2; ++y)
                for (int z = 0; z <= 2; ++z)
                    if (x + y + z == ord && (Q == 27 || x == 0 || y == 0 || z == 0)) b.m[n++] = MultiIndex{{x, y, z}};
    return b;
}

// 1-D population at velocity component c from the per-axis moment of order n.
constexpr double axis_inverse(int c, int n)
{
    if (c == 0) return n == 0 ? 1.0 : (n == 1 ? 0.0 : -1.0);
    return n == 0 ? 0.0 : (n == 1 ? 0.5 * c : 0.5);
}

// Per-axis moment of the weights (1, 0, c_s^2), i.e. of the rest state.
constexpr double axis_weight_moment(int n) { return n == 0 ? 1.0 : (n == 1 ? 0.0 : 1.0 / 3.0); }

constexpr int ipow(int c, int n) { return n == 0 ? 1 : (n == 1 ? c : c * c); }

template <int Q>
struct MB {
    static constexpr MomentBasis<Q> b = make_moment_basis<Q>();
    static constexpr int size = Q;
    static constexpr MultiIndex m(int j) { return b.m[j]; }
    static constexpr int n(int j, int a) { return b.m[j].n[a]; }
    static constexpr int ord(int j) { return order(b.m[j]); }
    static constexpr int find(int x, int y, int z)
    {
        for (int j = 0; j < Q; ++j)
            if (b.m[j].n[0] == x && b.m[j].n[1] == y && b.m[j].n[2] == z) return j;
        return -1;
    }
    // c_k^n
    static constexpr int mono(int j, int k)
    {
        return ipow(L<Q>::c(k, 0), n(j, 0)) * ipow(L<Q>::c(k, 1), n(j, 1)) * ipow(L<Q>::c(k, 2), n(j, 2));
    }
    // W_n = sum_k t_k c_k^n
    static constexpr double W(int j)
    {
        return axis_weight_moment(n(j, 0)) * axis_weight_moment(n(j, 1)) * axis_weight_moment(n(j, 2));
    }
    // Population k from raw moment j.
    static constexpr double inv(int k, int j)
    {
        return axis_inverse(L<Q>::c(k, 0), n(j, 0)) * axis_inverse(L<Q>::c(k, 1), n(j, 1)) *
               axis_inverse(L<Q>::c(k, 2), n(j, 2));
    }
    // i <= j componentwise
    static constexpr bool leq(int i, int j) { return n(i, 0) <= n(j, 0) && n(i, 1) <= n(j, 1) && n(i, 2) <= n(j, 2); }
    // prod_a C(n_a(j), n_a(i)) for i <= j
    static constexpr int binom(int j, int i)
    {
        int v = 1;
        for (int a = 0; a < 3; ++a) v *= (n(j, a) == 2 && n(i, a) == 1) ? 2 : 1;
        return v;
    }
    // Coefficient of moment i in the per-axis Hermite product of j:
    // h_2 = c^2 - c_s^2, so each axis of order 2 contributes 1 (order 2 kept)
    // or -1/3 (order 0); the inverse uses +1/3.
    static constexpr double hermite(int j, int i, double s)
    {
        double v = 1.0;
        for (int a = 0; a < 3; ++a) {
            if (n(i, a) == n(j, a)) continue;
            if (n(j, a) == 2 && n(i, a) == 0) v *= s;
            else return 0.0;
        }
        return v;
    }
};

template <int Q>
constexpr bool moment_inverse_is_exact()
{
    for (int k = 0; k < Q; ++k)
        for (int kk = 0; kk < Q; ++kk) {
            double s = 0.0;
            for (int j = 0; j < Q; ++j) s += MB<Q>::inv(k, j) * MB<Q>::mono(j, kk);
            if (s != (k == kk ? 1.0 : 0.0)) return false;
        }
    return true;
}
static_assert(moment_inverse_is_exact<19>(), "moment basis inverse");

// prod_a u_a^{e_a} for exponents e_a in {0,1,2}.
template <int EX, int EY, int EZ, class R>
__device__ __forceinline__ R upow(const R (&u)[3], const R (&u2)[3])
{
    R v = R(1);
    if constexpr (EX == 1) v *= u[0];
    if constexpr (EX == 2) v *= u2[0];
    if constexpr (EY == 1) v *= u[1];
    if constexpr (EY == 2) v *= u2[1];
    if constexpr (EZ == 1) v *= u[2];
    if constexpr (EZ == 2) v *= u2[2];
    return v;
}

// M^eq_n - W_n for the Maxwellian raw moments prod_a m_{n_a}, m = (1, u, u^2
// + c_s^2), accumulated axis by axis without forming a difference of O(1)
// numbers: with A the running deviation and B the running weight product,
// (A + B)(1/3 + u^2) - B/3 = A (1/3 + u^2) + B u^2.
template <int Q, int J, class R>
__device__ __forceinline__ R raw_eq_deviation(const R (&u)[3], const R (&u2)[3])
{
    using B = MB<Q>;
    R A = R(0);
    static_for<0, 3>([&](auto D) {
        constexpr int a = D;
        constexpr int na = B::n(J, a);
        constexpr double Bc = (a > 0 ? axis_weight_moment(B::n(J, 0)) : 1.0) *
                              (a > 1 ? axis_weight_moment(B::n(J, 1)) : 1.0);
        if constexpr (na == 1) {
            if constexpr (Bc != 0.0) A = (A + R(Bc)) * u[a];
            else A = A * u[a];
        } else if constexpr (na == 2) {
            if constexpr (Bc != 0.0) A = A * (R(1.0 / 3.0) + u2[a]) + R(Bc) * u2[a];
            else A = A * (R(1.0 / 3.0) + u2[a]);
        }
    });
    return A;
}

// Central non-equilibrium moments k_n - k_n^eq (k^eq = W for this basis) from
// the raw deviations dM: binomial expansion of prod_a (c_a - u_a)^{n_a}, with
// the rest-state part of every lower moment (W_i, i < n) added from constants.
template <int Q, int J, class R>
__device__ __forceinline__ R central_from_raw(const R (&dM)[Q], const R (&u)[3], const R (&u2)[3])
{
    using B = MB<Q>;
    R acc = dM[J];
    static_for<0, Q>([&](auto I) {
        constexpr int i = I;
        if constexpr (i != J && B::leq(i, J) && B::ord(i) >= 1) {
            constexpr int ex = B::n(J, 0) - B::n(i, 0), ey = B::n(J, 1) - B::n(i, 1), ez = B::n(J, 2) - B::n(i, 2);
            constexpr double cf = double(B::binom(J, i)) * (((ex + ey + ez) % 2) ? -1.0 : 1.0);
            acc += R(cf) * upow<ex, ey, ez>(u, u2) * dM[i];
        }
        if constexpr (i != J && B::leq(i, J) && B::W(i) != 0.0) {
            constexpr int ex = B::n(J, 0) - B::n(i, 0), ey = B::n(J, 1) - B::n(i, 1), ez = B::n(J, 2) - B::n(i, 2);
            constexpr double cf = double(B::binom(J, i)) * (((ex + ey + ez) % 2) ? -1.0 : 1.0) * B::W(i);
            acc += R(cf) * upow<ex, ey, ez>(u, u2);
        }
    });
    return acc;
}

// Raw change from a central change: prod_a c_a^{n_a} = prod_a ((c_a - u_a) +
// u_a)^{n_a}, the changes of orders 0 and 1 being zero.
template <int Q, int J, class R>
__device__ __forceinline__ R raw_from_central(const R (&dk)[Q], const R (&u)[3], const R (&u2)[3])
{
    using B = MB<Q>;
    R acc = dk[J];
    static_for<0, Q>([&](auto I) {
        constexpr int i = I;
        if constexpr (i != J && B::leq(i, J) && B::ord(i) >= 2) {
            constexpr int ex = B::n(J, 0) - B::n(i, 0), ey = B::n(J, 1) - B::n(i, 1), ez = B::n(J, 2) - B::n(i, 2);
            acc += R(double(B::binom(J, i))) * upow<ex, ey, ez>(u, u2) * dk[i];
        }
    });
    return acc;
}

// Hermite image (SIGN = -1: h_2 = c^2 - 1/3 per axis) or its inverse (SIGN =
// +1: c^2 = h_2 + 1/3) of moment J, using the moments of order >= LOWEST.
template <int Q, int J, int LOWEST, int SIGN, class R>
__device__ __forceinline__ R hermite_map(const R (&x)[Q])
{
    using B = MB<Q>;
    R acc = x[J];
    static_for<0, Q>([&](auto I) {
        constexpr int i = I;
        if constexpr (i != J && B::ord(i) >= LOWEST) {
            constexpr double cf = B::hermite(J, i, SIGN * (1.0 / 3.0));
            if constexpr (cf != 0.0) acc += R(cf) * x[i];
        }
    });
    return acc;
}

enum MomentFamily { FAM_RAW = 0, FAM_HERMITE = 1, FAM_CENTRAL = 2, FAM_CHERMITE = 3 };

template <class R>
struct MomentRates {
    R w, wp, wm, w3, w4;  // shear, Eq. bulk mixing (w+, w-), third order, order >= 4
};

// Change of the relaxed moment J of order >= 2 (Eq. RMcoll, Eq. bulk).
template <int Q, int J, class R>
__device__ __forceinline__ R relax_change(const R (&N)[Q], const MomentRates<R>& r)
{
    using B = MB<Q>;
    constexpr int o = B::ord(J);
    constexpr bool diag = o == 2 && (B::n(J, 0) == 2 || B::n(J, 1) == 2 || B::n(J, 2) == 2);
    if constexpr (diag) {
        constexpr int a = B::n(J, 0) == 2 ? 0 : (B::n(J, 1) == 2 ? 1 : 2);
        constexpr int x1 = a == 0 ? B::find(0, 2, 0) : B::find(2, 0, 0);
        constexpr int x2 = a == 2 ? B::find(0, 2, 0) : B::find(0, 0, 2);
        static_assert(x1 >= 0 && x2 >= 0, "second-order basis");
        return -(r.wp * N[J] + r.wm * (N[x1] + N[x2]));
    } else if constexpr (o == 2) {
        return -r.w * N[J];
    } else if constexpr (o == 3) {
        return -r.w3 * N[J];
    } else {
        return -r.w4 * N[J];
    }
}

// One cell of a moment-space model; g in the storage representation (shifted
// or not), m its pair sums and macroscopic values. NW4 is the raw-moment
// model with every rate equal to omega.
template <int Q, int FAM, bool CUMULANT, class R>
__device__ __forceinline__ void collide_moment_space(R (&g)[Q], const R (&s)[L<Q>::half], const R (&d)[L<Q>::half],
                                                     R base, R rho, const R (&u)[3], const MomentRates<R>& r)
{
    using S = L<Q>;
    using B = MB<Q>;
    static_assert(!CUMULANT || Q == 19, "cumulant model on D3Q19");
    const R inv_rho = R(1) / rho;
    const R u2[3] = {u[0] * u[0], u[1] * u[1], u[2] * u[2]};

    // Raw deviations dM_n = M_n - W_n (orders 0 and 1: 0 and u).
    R dM[Q];
    static_for<0, Q>([&](auto J) {
        constexpr int j = J;
        if constexpr (B::ord(j) == 0) {
            dM[j] = R(0);
        } else if constexpr (B::ord(j) == 1) {
            dM[j] = u[B::n(j, 0) ? 0 : (B::n(j, 1) ? 1 : 2)];
        } else {
            R acc = R(0);
            static_for<0, S::half>([&](auto K) {
                constexpr int k = K;
                constexpr int c = B::mono(j, k);
                if constexpr (B::ord(j) % 2 == 0) {
                    if constexpr (c == 1) acc += s[k];
                    else if constexpr (c == -1) acc -= s[k];
                } else {
                    if constexpr (c == 1) acc += d[k];
                    else if constexpr (c == -1) acc -= d[k];
                }
            });
            if constexpr (B::W(j) != 0.0) acc -= R(B::W(j)) * base;
            dM[j] = acc * inv_rho;
        }
    });

    // Non-equilibrium moments N_n = X_n - X_n^eq of the family (orders >= 2).
    R N[Q];
    static_for<0, Q>([&](auto J) {
        constexpr int j = J;
        if constexpr (B::ord(j) < 2) {
            N[j] = R(0);
        } else if constexpr (FAM == FAM_RAW) {
            N[j] = dM[j] - raw_eq_deviation<Q, j>(u, u2);
        } else if constexpr (FAM == FAM_HERMITE) {
            N[j] = hermite_map<Q, j, 1, -1>(dM) - upow<B::n(j, 0), B::n(j, 1), B::n(j, 2)>(u, u2);
        } else {
            N[j] = central_from_raw<Q, j>(dM, u, u2);
        }
    });
    if constexpr (FAM == FAM_CHERMITE) {
        R C[Q];
        static_for<0, Q>([&](auto J) {
            constexpr int j = J;
            C[j] = B::ord(j) < 2 ? R(0) : hermite_map<Q, j, 2, -1>(N);
        });
        static_for<0, Q>([&](auto J) { N[J] = C[J]; });
    }

    // Relaxation: dX_n = X*_n - X_n.
    R dX[Q];
    static_for<0, Q>([&](auto J) {
        constexpr int j = J;
        if constexpr (B::ord(j) < 2) dX[j] = R(0);
        else dX[j] = relax_change<Q, j>(N, r);
    });
    if constexpr (CUMULANT) {
        // Fourth order: C_aabb = k_aabb - k_aa k_bb - 2 k_ab^2 relaxes to
        // (1 - w4) C_aabb; with k = k^eq + N, k^eq_aa = 1/3, k^eq_aabb = 1/9.
        static_for<0, 3>([&](auto P) {
            constexpr int p = P;
            constexpr int a = p == 2 ? 1 : 0, b = p == 0 ? 1 : 2;
            constexpr int i4 = B::find(a == 0 ? 2 : 0, (a == 1 || b == 1) ? 2 : 0, b == 2 ? 2 : 0);
            constexpr int ia = B::find(a == 0 ? 2 : 0, a == 1 ? 2 : 0, 0);
            constexpr int ib = B::find(0, b == 1 ? 2 : 0, b == 2 ? 2 : 0);
            constexpr int iab = B::find(a == 0 ? 1 : 0, (a == 1 || b == 1) ? 1 : 0, b == 2 ? 1 : 0);
            static_assert(i4 >= 0 && ia >= 0 && ib >= 0 && iab >= 0, "fourth-order cumulant indices");
            const R third = R(1.0 / 3.0);
            const R C = N[i4] - third * (N[ia] + N[ib]) - N[ia] * N[ib] - R(2) * N[iab] * N[iab];
            const R Na = N[ia] + dX[ia], Nb = N[ib] + dX[ib], Nab = N[iab] + dX[iab];
            const R N4 = (R(1) - r.w4) * C + third * (Na + Nb) + Na * Nb + R(2) * Nab * Nab;
            dX[i4] = N4 - N[i4];
        });
    }

    // Back to raw changes dM*_n - dM_n.
    R dR[Q];
    if constexpr (FAM == FAM_RAW) {
        static_for<0, Q>([&](auto J) { dR[J] = dX[J]; });
    } else if constexpr (FAM == FAM_HERMITE) {
        static_for<0, Q>([&](auto J) {
            constexpr int j = J;
            dR[j] = B::ord(j) < 2 ? R(0) : hermite_map<Q, j, 2, 1>(dX);
        });
    } else {
        R dk[Q];
        if constexpr (FAM == FAM_CHERMITE) {
            static_for<0, Q>([&](auto J) {
                constexpr int j = J;
                dk[j] = B::ord(j) < 2 ? R(0) : hermite_map<Q, j, 2, 1>(dX);
            });
        } else {
            static_for<0, Q>([&](auto J) { dk[J] = dX[J]; });
        }
        static_for<0, Q>([&](auto J) {
            constexpr int j = J;
            dR[j] = B::ord(j) < 2 ? R(0) : raw_from_central<Q, j>(dk, u, u2);
        });
    }

    // Populations: g_k += rho sum_n Minv[k][n] dR_n, split into the parts even
    // and odd in c so that k and k-bar share one evaluation.
    static_for<0, S::half + 1>([&](auto K) {
        constexpr int k = K;
        R ev = R(0), od = R(0);
        static_for<0, Q>([&](auto J) {
            constexpr int j = J;
            constexpr double cf = B::inv(k, j);
            if constexpr (B::ord(j) >= 2 && cf != 0.0) {
                if constexpr (B::ord(j) % 2 == 0) ev += R(cf) * dR[j];
                else od += R(cf) * dR[j];
            }
        });
        if constexpr (k == S::rest) {
            g[k] += rho * ev;
        } else {
            g[k] += rho * (ev + od);
            g[S::opp(k)] += rho * (ev - od);
        }
    });
}

// NW4 equilibrium in the storage representation: f^eq = rho Minv M^eq with
// Minv W = t, so f^eq_k - shift t_k = base t_k + rho sum_n Minv[k][n] (M^eq_n
// - W_n), base = rho - shift.
template <int Q, class R>
__device__ __forceinline__ void equilibrium_nw4(R base, R rho, const R (&u)[3], R (&g)[Q])
{
    using S = L<Q>;
    using B = MB<Q>;
    const R u2[3] = {u[0] * u[0], u[1] * u[1], u[2] * u[2]};
    R P[Q];
    static_for<0, Q>([&](auto J) {
        constexpr int j = J;
        P[j] = B::ord(j) == 0 ? R(0) : raw_eq_deviation<Q, j>(u, u2);
    });
    static_for<0, S::half + 1>([&](auto K) {
        constexpr int k = K;
        R ev = R(0), od = R(0);
        static_for<0, Q>([&](auto J) {
            constexpr int j = J;
            constexpr double cf = B::inv(k, j);
            if constexpr (B::ord(j) >= 1 && cf != 0.0) {
                if constexpr (B::ord(j) % 2 == 0) ev += R(cf) * P[j];
                else od += R(cf) * P[j];
            }
        });
        const R tb = R(S::t(k)) * base;
        if constexpr (k == S::rest) {
            g[k] = tb + rho * ev;
        } else {
            g[k] = tb + rho * (ev + od);
            g[S::opp(k)] = tb + rho * (ev - od);
        }
    });
}

}  // namespace lbm
