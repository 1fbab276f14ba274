// dsim_ncp.h -- the frictional-contact NCP (Section II.B, eq. NCP) and the
// reduced implicit system of its mode split (Section III.B-C, Appendix B).
//
// Solve: block Gauss-Seidel sweeps with exact per-contact solves (working
// precision), then Newton on the equations of the realised modes (FP64) with
// active-set changes; the natural-map residual is checked in FP64.  The
// paper's reduced matrix A is then formed at the solution and factorised in
// FP64 for the derivative.
#pragma once

#include "dsim_core.h"

namespace dsim {

// Iteration caps of the solve's fallback pass: damped Newton on the
// natural map, ADMM.
constexpr int kLmIters = 40;
constexpr int kAdmmIters = 1500;

// Unit slip direction t solving (s I + r Wt) t = bt for s > 0, with Wt given
// by its eigen-decomposition (l1 >= l2 >= 0, unit eigenvector (e0, e1) of l1)
// and bt by its coordinates beta in that basis.  |t(s)| decreases in s;
// Newton on 1/|t(s)| = 1 (the trust-region secular equation).
template <class R>
DSIM_HD inline void slip_direction(R l1, R l2, R e0, R e1, R beta1, R beta2, R r, R& t0, R& t1) {
    const R p1 = r * l1, p2 = r * (l2 > R(0) ? l2 : R(0));
    const R tiny = R(1e-30);
    R sv = 0;
    if (p2 <= R(1e-12) * (p1 + tiny)) sv = fabs(beta2);
    if (p1 + sv <= tiny) sv = fabs(beta1) + fabs(beta2);
    for (int it = 0; it < 40; ++it) {
        const R d1 = sv + p1, d2 = sv + p2;
        const R q1 = beta1 / d1, q2 = d2 > tiny ? beta2 / d2 : R(0);
        const R n2 = q1 * q1 + q2 * q2;
        const R nrm = sqrt(n2);
        if (!(nrm > R(0))) break;
        const R psi = R(1) / nrm - R(1);
        const R dn2 = q1 * q1 / d1 + (d2 > tiny ? q2 * q2 / d2 : R(0));
        const R dpsi = dn2 / (n2 * nrm);
        if (!(dpsi > R(0))) break;
        R sn = sv - psi / dpsi;
        if (sn <= R(0)) sn = R(0.5) * sv;
        const R ds = fabs(sn - sv);
        sv = sn;
        // FP32 stops at 1e-6 relative: closer to its rounding unit the step
        // only oscillates until the iteration cap
        if (ds <= R(sizeof(R) == 4 ? 1e-6 : 9.2e-16) * (sv + p1)) break;
    }
    const R d1 = sv + p1, d2 = sv + p2;
    const R q1 = d1 > tiny ? beta1 / d1 : R(0), q2 = d2 > tiny ? beta2 / d2 : R(0);
    const R u0 = e0 * q1 - e1 * q2, u1 = e1 * q1 + e0 * q2;
    const R nu = sqrt(u0 * u0 + u1 * u1);
    if (nu > R(0)) {
        t0 = u0 / nu;
        t1 = u1 / nu;
    } else {
        t0 = 1;
        t1 = 0;
    }
}

// One-contact problem sigma = W Lam + b.  Separation if the normal free
// velocity is non-negative, else the sticking impulse if it lies in the
// cone, else the sliding impulse on the cone boundary.
//
// Sliding: sigma_N = 0 gives Lam_N = -(b_N + W_NT . Lam_T) / W_NN, so
// sigma_T = Wt Lam_T + bt with the Schur complement Wt = W_TT - W_TN W_NT^T / W_NN
// and bt = b_T - W_TN b_N / W_NN.  With Lam_T = -r t (|t| = 1, r = mu Lam_N)
// and sigma_T = s t (s > 0):  (s I + r Wt) t = bt, which fixes t(r); r itself
// solves g(r) = r (W_NN - mu W_NT . t(r)) + mu b_N = 0, with g(0) = mu b_N < 0:
// bracketed, then refined by regula falsi (Illinois variant).
// Sliding impulse of one contact by Newton's method from a warm start
// (the previous sliding impulse): unknowns Lam, equations
// Lam_T + mu Lam_N u(sigma_T) = 0 and sigma_N = 0 with sigma = W Lam + b.
// Returns false if it does not converge to a consistent sliding impulse.
template <class R>
DSIM_HD inline bool slide_newton(const R* W, const R* b, R mu, R* lam) {
    R L0 = lam[0], L1 = lam[1], L2 = lam[2];
    const R tol = R(sizeof(R) == 4 ? 2e-6 : 1e-13);
    for (int it = 0; it < 6; ++it) {
        const R s0 = W[0] * L0 + W[1] * L1 + W[2] * L2 + b[0];
        const R s1 = W[3] * L0 + W[4] * L1 + W[5] * L2 + b[1];
        const R s2 = W[6] * L0 + W[7] * L1 + W[8] * L2 + b[2];
        const R ns = sqrt(s0 * s0 + s1 * s1);
        if (!(ns > R(0)) || !(L2 > R(0))) return false;
        const R u0 = s0 / ns, u1 = s1 / ns;
        const R f0 = L0 + mu * L2 * u0, f1 = L1 + mu * L2 * u1, f2 = s2;
        const R lsc = mu * L2 + fabs(L0) + fabs(L1);
        const R ssc = fabs(b[2]) + ns;
        if (fabs(f0) <= tol * lsc && fabs(f1) <= tol * lsc && fabs(f2) <= tol * ssc) {
            lam[0] = L0;
            lam[1] = L1;
            lam[2] = L2;
            return (L0 * s0 + L1 * s1) < R(0);
        }
        // Jacobian rows: tangential e_a + mu u_a e_N + (mu L_N/|s_T|) (I - u u^T)_a W_T,
        // normal W_N
        const R c = mu * L2 / ns;
        const R h00 = 1 - u0 * u0, h01 = -u0 * u1, h11 = 1 - u1 * u1;
        R Jm[9];
        for (int j = 0; j < 3; ++j) {
            Jm[j] = c * (h00 * W[j] + h01 * W[3 + j]);
            Jm[3 + j] = c * (h01 * W[j] + h11 * W[3 + j]);
            Jm[6 + j] = W[6 + j];
        }
        Jm[0] += 1;
        Jm[4] += 1;
        Jm[2] += mu * u0;
        Jm[5] += mu * u1;
        const R c00 = Jm[4] * Jm[8] - Jm[5] * Jm[7], c01 = Jm[5] * Jm[6] - Jm[3] * Jm[8],
                c02 = Jm[3] * Jm[7] - Jm[4] * Jm[6];
        const R det = Jm[0] * c00 + Jm[1] * c01 + Jm[2] * c02;
        // a (numerically) singular Jacobian: the impulse is not determined
        // along some direction, and a Newton step along it is unbounded
        R rn[3];
        for (int i = 0; i < 3; ++i)
            rn[i] = fabs(Jm[3 * i]) + fabs(Jm[3 * i + 1]) + fabs(Jm[3 * i + 2]);
        if (!(fabs(det) > R(sizeof(R) == 4 ? 1e-6 : 1e-12) * rn[0] * rn[1] * rn[2])) return false;
        const R id = R(1) / det;
        // step = -J^-1 f (adjugate)
        const R d0 = -(c00 * f0 + (Jm[2] * Jm[7] - Jm[1] * Jm[8]) * f1 + (Jm[1] * Jm[5] - Jm[2] * Jm[4]) * f2) * id;
        const R d1 = -(c01 * f0 + (Jm[0] * Jm[8] - Jm[2] * Jm[6]) * f1 + (Jm[2] * Jm[3] - Jm[0] * Jm[5]) * f2) * id;
        const R d2 = -(c02 * f0 + (Jm[1] * Jm[6] - Jm[0] * Jm[7]) * f1 + (Jm[0] * Jm[4] - Jm[1] * Jm[3]) * f2) * id;
        L0 += d0;
        L1 += d1;
        L2 += d2;
    }
    return false;
}

template <class R>
DSIM_HD inline int local_solve(const R* W, const R* Wi, const R* b, R mu, R* lam, int prev_mode) {
    // separating, or a point whose normal velocity no impulse changes (its
    // normal row of the block is zero up to rounding)
    if (b[2] >= R(0) || !(W[8] > R(sizeof(R) == 4 ? 1e-6 : 1e-12) * (W[0] + W[4] + W[8]))) {
        lam[0] = lam[1] = lam[2] = 0;
        return BRK;
    }
    R s[3];
    mat3vec(Wi, b, s);
    s[0] = -s[0]; s[1] = -s[1]; s[2] = -s[2];
    const R nt = sqrt(s[0] * s[0] + s[1] * s[1]);
    if (s[2] > R(0) && nt <= mu * s[2]) {
        lam[0] = s[0]; lam[1] = s[1]; lam[2] = s[2];
        return STK;
    }
    if (prev_mode == SLD && mu > R(0) && slide_newton(W, b, mu, lam)) return SLD;
    const R wnn = W[8];
    if (mu <= R(0) || !(wnn > R(0))) {
        lam[0] = 0;
        lam[1] = 0;
        lam[2] = wnn > R(0) ? -b[2] / wnn : R(0);
        return SLD;
    }
    const R w00 = W[0] - W[2] * W[6] / wnn;
    const R w11 = W[4] - W[5] * W[7] / wnn;
    const R w01 = R(0.5) * ((W[1] - W[2] * W[7] / wnn) + (W[3] - W[5] * W[6] / wnn));
    const R bt0 = b[0] - W[2] * b[2] / wnn, bt1 = b[1] - W[5] * b[2] / wnn;
    // eigen-decomposition of the symmetric 2x2 Wt; (e0, e1) is the larger of
    // (l1 - w11, w01) and (w01, l1 - w00), both solutions of (Wt - l1 I) e = 0
    const R disc = sqrt(R(0.25) * (w00 - w11) * (w00 - w11) + w01 * w01);
    const R l1 = R(0.5) * (w00 + w11) + disc, l2 = R(0.5) * (w00 + w11) - disc;
    R e0 = l1 - w11, e1 = w01;
    {
        const R f0 = w01, f1 = l1 - w00;
        if (f0 * f0 + f1 * f1 > e0 * e0 + e1 * e1) {
            e0 = f0;
            e1 = f1;
        }
        const R nn = sqrt(e0 * e0 + e1 * e1);
        if (nn > R(0)) {
            e0 /= nn;
            e1 /= nn;
        } else {
            e0 = 1;
            e1 = 0;
        }
    }
    const R beta1 = e0 * bt0 + e1 * bt1, beta2 = -e1 * bt0 + e0 * bt1;
    R t0 = 1, t1 = 0;
    auto gfun = [&](R r) -> R {
        slip_direction(l1, l2, e0, e1, beta1, beta2, r, t0, t1);
        return r * (wnn - mu * (W[6] * t0 + W[7] * t1)) + mu * b[2];
    };
    R rlo = 0, glo = mu * b[2];
    R rhi = -mu * b[2] / wnn, ghi = gfun(rhi);
    for (int it = 0; it < 60 && !(ghi > R(0)); ++it) {
        rlo = rhi;
        glo = ghi;
        rhi *= R(2);
        ghi = gfun(rhi);
    }
    if (!(ghi > R(0))) {
        // no sliding impulse makes the normal velocity vanish (a singular
        // block): the sticking candidate pulled radially onto the cone
        const R sn = s[2] > R(0) ? s[2] : R(0);
        const R f = (nt > mu * sn && nt > R(0)) ? mu * sn / nt : R(1);
        lam[0] = s[0] * f;
        lam[1] = s[1] * f;
        lam[2] = sn;
        return sn > R(0) ? SLD : BRK;
    }
    R r = rhi;
    {
        int side = 0;
        // bracket width at which the search stops; in FP32 a width near the
        // rounding unit is rarely reached and the search would run to its cap
        // (the refinement that follows works in FP64 anyway)
        const R rtol = R(sizeof(R) == 4 ? 1e-6 : 1e-15);
        for (int it = 0; it < 100; ++it) {
            r = (rlo * ghi - rhi * glo) / (ghi - glo);
            if (!(r > rlo && r < rhi)) r = R(0.5) * (rlo + rhi);
            const R gr = gfun(r);
            if (gr > R(0)) {
                rhi = r;
                ghi = gr;
                if (side == 1) glo *= R(0.5);
                side = 1;
            } else {
                rlo = r;
                glo = gr;
                if (side == -1) ghi *= R(0.5);
                side = -1;
            }
            if (rhi - rlo <= rtol * rhi || gr == R(0)) break;
        }
    }
    gfun(r);
    lam[0] = -r * t0;
    lam[1] = -r * t1;
    lam[2] = r / mu;
    return SLD;
}

// At most `sweeps` block Gauss-Seidel sweeps, run by wavefront 0: sigma =
// G Lam + g is kept up to date in LDS; each contact update is computed
// redundantly by all lanes, then the lanes update sigma row-parallel.  G in
// working precision is the rounding of the FP64 Delassus matrix, taken from
// Gd as it is read (no second copy on chip).  A
// sweep that changes no impulse and no mode has reached a fixed point in
// working precision: every further sweep would repeat it exactly, so the
// sweeps end there (the same result as running them all).
template <class R>
DSIM_HD void nsgs(const Team& T, Env<R>& E, int sweeps) {
    const int k = E.k, nc = E.nc;
    if (T.wave == 0) {
        for (int s = 0; s < sweeps; ++s) {
            bool moved = false;  // uniform over the wavefront
            for (int c = 0; c < nc; ++c) {
                const int o = 3 * c;
                R W[9];
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) W[3 * i + j] = R(E.Gd[(o + i) * k + o + j]);
                const R L[3] = {E.Lam[o], E.Lam[o + 1], E.Lam[o + 2]};
                R b[3];
                for (int i = 0; i < 3; ++i)
                    b[i] = E.sig[o + i] - (W[3 * i] * L[0] + W[3 * i + 1] * L[1] + W[3 * i + 2] * L[2]);
                R Ln[3] = {L[0], L[1], L[2]};
                const int prev = E.lmode[c];
                const int md = local_solve(W, E.Winv + 9 * c, b, E.mu[c], Ln, prev);
                const R d0 = Ln[0] - L[0], d1 = Ln[1] - L[1], d2 = Ln[2] - L[2];
                // NaN differences compare unequal to zero and keep sweeping
                moved = moved || md != prev || !(d0 == R(0) && d1 == R(0) && d2 == R(0));
                T.wave_sync();
                for (int r = T.lane; r < k; r += T.wsize)
                    E.sig[r] += R(E.Gd[r * k + o]) * d0 + R(E.Gd[r * k + o + 1]) * d1 + R(E.Gd[r * k + o + 2]) * d2;
                if (T.lane == 0) {
                    E.Lam[o] = Ln[0];
                    E.Lam[o + 1] = Ln[1];
                    E.Lam[o + 2] = Ln[2];
                    E.lmode[c] = md;
                }
                T.wave_sync();
            }
            if (T.lane == 0) E.hdr[7] += 1;  // sweeps executed
            if (!moved) break;
        }
    }
    T.sync();
}

// sigma = Gd Ld + gd in FP64.
template <class R, class TT>
DSIM_HD void fp64_sigma(const TT& T, Env<R>& E) {
    const int k = E.k;
    for (int r = T.tid; r < k; r += T.nt) {
        double s = E.gd[r];
        for (int c = 0; c < k; ++c) s += E.Gd[r * k + c] * E.Ld[c];
        E.dsig[r] = s;
    }
    T.sync();
}

// Scales of the residuals: free velocity (with the gravity step) and impulse.
template <class R>
DSIM_HD inline void scales(const Env<R>& E, const Params& P, double& smax, double& lmax) {
    smax = 1e-300;
    lmax = 1e-300;
    for (int r = 0; r < E.k; ++r) {
        const double a = fabs(E.gd[r]);
        smax = a > smax ? a : smax;
        const double l = fabs(E.Ld[r]);
        lmax = l > lmax ? l : lmax;
    }
    const double sg = P.dt * (fabs(P.gx) + fabs(P.gy) + fabs(P.gz));
    smax = smax > sg ? smax : sg;
}

// Reduced variables of the mode set in cmode (Section III.C, Appendix B):
// sticking contacts first (3 each), then sliding contacts (2 each, in the
// tangent plane of the cone, R = [Lam/|Lam|, e_z x sigma_T/|sigma_T|]).  Row
// vectors select the equation rows; the sliding rows are scaled so that the
// coefficients stay bounded: the first by 1/cos(phi) (row e_z), the second by
// alpha/(1 + alpha) (row w u_perp, diagonal 1 - w, w = mu Lam_N / (mu Lam_N +
// |sigma_T|)).  Uses Ld and dsig.
template <class R>
DSIM_HD void reduced_vars(const Team& T, Env<R>& E) {
    if (T.tid == 0) {
        int m = 0, nstk = 0;
        for (int pass = 0; pass < 2; ++pass)
            for (int c = 0; c < E.nc; ++c) {
                const int md = E.cmode[c];
                if (pass == 0 && md == STK) {
                    for (int a = 0; a < 3; ++a) {
                        E.vctc[m] = c;
                        E.vcmp[m] = a;
                        for (int i = 0; i < 3; ++i) {
                            E.vrow[3 * m + i] = (i == a) ? 1.0 : 0.0;
                            E.vcol[3 * m + i] = (i == a) ? 1.0 : 0.0;
                        }
                        E.vdiag[m] = 0;
                        ++m;
                    }
                    ++nstk;
                } else if (pass == 1 && md == SLD) {
                    const int o = 3 * c;
                    const double s0 = E.dsig[o], s1 = E.dsig[o + 1];
                    const double ns = sqrt(s0 * s0 + s1 * s1);
                    const double u0 = ns > 0 ? s0 / ns : 1.0, u1 = ns > 0 ? s1 / ns : 0.0;
                    const double L0 = E.Ld[o], L1 = E.Ld[o + 1], L2 = E.Ld[o + 2];
                    const double nl = sqrt(L0 * L0 + L1 * L1 + L2 * L2);
                    const double mln = double(E.mu[c]) * L2;
                    const double w = (mln + ns) > 0 ? mln / (mln + ns) : 1.0;
                    // along r1 = Lam/|Lam|: row e_z
                    E.vctc[m] = c;
                    E.vcmp[m] = 0;
                    E.vrow[3 * m] = 0;
                    E.vrow[3 * m + 1] = 0;
                    E.vrow[3 * m + 2] = 1;
                    E.vcol[3 * m] = L0 / nl;
                    E.vcol[3 * m + 1] = L1 / nl;
                    E.vcol[3 * m + 2] = L2 / nl;
                    E.vdiag[m] = 0;
                    ++m;
                    // along r2 = e_z x u: row w u_perp, diagonal 1 - w
                    E.vctc[m] = c;
                    E.vcmp[m] = 1;
                    E.vrow[3 * m] = -w * u1;
                    E.vrow[3 * m + 1] = w * u0;
                    E.vrow[3 * m + 2] = 0;
                    E.vcol[3 * m] = -u1;
                    E.vcol[3 * m + 1] = u0;
                    E.vcol[3 * m + 2] = 0;
                    E.vdiag[m] = 1 - w;
                    ++m;
                }
            }
        E.hdr[1] = m;
        E.hdr[2] = nstk;
    }
    T.sync();
}

// A = rows^T G cols + diag (FP64), m x m row-major.
template <class R>
DSIM_HD void build_A(const Team& T, Env<R>& E) {
    const int m = E.hdr[1], k = E.k;
    for (int idx = T.tid; idx < m * m; idx += T.nt) {
        const int i = idx / m, j = idx - i * m;
        const int ci = 3 * E.vctc[i], cj = 3 * E.vctc[j];
        const double* ri = E.vrow + 3 * i;
        const double* cv = E.vcol + 3 * j;
        double s = 0;
        for (int a = 0; a < 3; ++a) {
            if (ri[a] == 0.0) continue;
            double t = 0;
            for (int b = 0; b < 3; ++b) t += E.Gd[(ci + a) * k + cj + b] * cv[b];
            s += ri[a] * t;
        }
        if (i == j) s += E.vdiag[i];
        E.A[idx] = s;
    }
    T.sync();
}

// In-place elimination of A with pivoting.  Sticking variables come first
// and are eliminated with symmetric (diagonal) pivoting: that block is G_SS,
// symmetric positive semidefinite, so this is a pivoted LDL^T (square-root
// free Cholesky) of it.  Once it is exhausted the elimination continues with
// complete pivoting (the sliding block's Schur complement; the remaining
// sticking rows and columns are zero).  Pivots below rank_tol times the
// largest entry of A end the elimination; the solves then set the remaining
// variables to zero (basic solution).  Leaves L (unit, below the diagonal)
// and U in A, the row and column permutations in rperm/cperm, the rank in
// hdr[4].
template <class R, class TT>
DSIM_INLINE DSIM_HD void factor_A(const TT& T, Env<R>& E, double rank_tol) {
    const int m = E.hdr[1];
    const int nst = 3 * E.hdr[2];
    double* A = E.A;
    for (int i = T.tid; i < m; i += T.nt) {
        E.rperm[i] = i;
        E.cperm[i] = i;
    }
    // largest entry (a team reduction; the index is unused)
    double scale = -1;
    int si = INT_MAX;
    for (int idx = T.tid; idx < m * m; idx += T.nt) {
        const double a = fabs(A[idx]);
        if (a > scale) {
            scale = a;
            si = idx;
        }
    }
    team_argmax(T, E.redv, E.redi, scale, si);
    T.sync();
    const double tol = rank_tol * (scale > 0 ? scale : 1.0);
    int rank = 0;
    bool stick_phase = nst > 0;
    for (int p = 0; p < m; ++p) {
        // pivot choice: a strided scan per thread, then the team maximum
        // (first maximum in index order, as one serial scan would find)
        int pr = -1, pc = -1;
        double best = -1;
        int bi = INT_MAX;
        if (stick_phase && p < nst) {
            for (int i = p + T.tid; i < nst; i += T.nt) {
                const double a = fabs(A[i * m + i]);
                if (a > best) {
                    best = a;
                    bi = i;
                }
            }
            team_argmax(T, E.redv, E.redi, best, bi);
            if (bi != INT_MAX) {
                pr = bi;
                pc = bi;
            }
            if (best <= tol) {
                stick_phase = false;
                T.sync();  // the reduction slots are reused below
            }
        }
        if (!(stick_phase && p < nst)) {
            best = -1;
            bi = INT_MAX;
            const int rem = m - p;
            for (int idx = T.tid; idx < rem * rem; idx += T.nt) {
                const int i = p + idx / rem, j = p + idx % rem;
                const double a = fabs(A[i * m + j]);
                if (a > best) {
                    best = a;
                    bi = i * m + j;
                }
            }
            team_argmax(T, E.redv, E.redi, best, bi);
            pr = -1;
            pc = -1;
            if (bi != INT_MAX) {
                pr = bi / m;
                pc = bi - pr * m;
            }
        }
        if (best <= tol || pr < 0) break;
        T.sync();
        if (pr != p)
            for (int j = T.tid; j < m; j += T.nt) {
                const double t = A[p * m + j];
                A[p * m + j] = A[pr * m + j];
                A[pr * m + j] = t;
            }
        T.sync();
        if (pc != p)
            for (int i = T.tid; i < m; i += T.nt) {
                const double t = A[i * m + p];
                A[i * m + p] = A[i * m + pc];
                A[i * m + pc] = t;
            }
        if (T.tid == 0) {
            int t = E.rperm[p];
            E.rperm[p] = E.rperm[pr];
            E.rperm[pr] = t;
            t = E.cperm[p];
            E.cperm[p] = E.cperm[pc];
            E.cperm[pc] = t;
        }
        T.sync();
        const double piv = A[p * m + p];
        for (int i = p + 1 + T.tid; i < m; i += T.nt) A[i * m + p] /= piv;
        T.sync();
        const int rem = m - p - 1;
        for (int idx = T.tid; idx < rem * rem; idx += T.nt) {
            const int i = p + 1 + idx / rem, j = p + 1 + idx % rem;
            A[i * m + j] -= A[i * m + p] * A[p * m + j];
        }
        T.sync();
        rank = p + 1;
    }
    if (T.tid == 0) E.hdr[4] = rank;
    T.sync();
}

// Solve A x = b with the factors for one right-hand side (basic solution):
// b permuted by rperm, free variables zero, result scattered by cperm.
DSIM_HD inline void lu_solve(const double* A, int m, int rank, const int* rperm, const int* cperm,
                             const double* b, double* y, double* x) {
    for (int i = 0; i < m; ++i) y[i] = b[rperm[i]];
    for (int i = 0; i < rank; ++i) {
        double s = y[i];
        for (int j = 0; j < i; ++j) s -= A[i * m + j] * y[j];
        y[i] = s;
    }
    for (int i = rank; i < m; ++i) y[i] = 0;
    for (int i = rank - 1; i >= 0; --i) {
        double s = y[i];
        for (int j = i + 1; j < rank; ++j) s -= A[i * m + j] * y[j];
        y[i] = s / A[i * m + i];
    }
    for (int i = 0; i < m; ++i) x[cperm[i]] = y[i];
}

// lu_solve on wavefront 0: lane r keeps y_r in a register; the forward and
// back substitutions go column by column, broadcasting each finished y_i
// with a cross-lane shuffle (m <= 63).  The host build runs lu_solve.
DSIM_HD inline void wave_lu_solve(const Team& T, const double* A, int m, int rank, const int* rperm,
                                  const int* cperm, const double* b, double* y, double* x) {
#ifdef DSIM_HOST_BUILD
    lu_solve(A, m, rank, rperm, cperm, b, y, x);
#else
    (void)y;
    const int r = T.lane;
    double yr = r < m ? b[rperm[r]] : 0.0;
    for (int i = 0; i < rank; ++i) {
        const double yi = __shfl(yr, i, 64);
        if (r > i && r < rank) yr -= A[r * m + i] * yi;
    }
    if (r >= rank) yr = 0.0;
    for (int i = rank - 1; i >= 0; --i) {
        const double yi = __shfl(yr, i, 64) / A[i * m + i];
        if (r == i)
            yr = yi;
        else if (r < i)
            yr -= A[r * m + i] * yi;
    }
    if (r < m) x[cperm[r]] = yr;
    T.wave_sync();
#endif
}

// Newton system of the mode equations (Section III.B) in the impulses of the
// active contacts (3 unknowns each, sticking contacts first): sticking
// sigma_c = 0; sliding Lam_T + mu Lam_N u = 0 (u = sigma_T/|sigma_T|) and
// sigma_N = 0.  Fills A (its exact Jacobian), rhs = -F and the unknowns'
// contact and component; dsc[1] gets the scaled residual max |F_i| / scale
// and dsc[3] its squared 2-norm (velocity rows scaled by the free-velocity
// scale, impulse rows by the impulse scale).  Uses Ld and dsig.
template <class R, class TT>
DSIM_INLINE DSIM_HD void newton_system(const TT& T, Env<R>& E, const Params& P) {
    const int k = E.k, nc = E.nc;
    // unknowns: every thread counts the active contacts (sticking first,
    // then sliding) and thread c fills the slots of contact c
    int nstk = 0, nact = 0;
    for (int c = 0; c < nc; ++c) {
        const int md = E.cmode[c];
        nstk += md == STK;
        nact += md != BRK;
    }
    const int m = 3 * nact;
    for (int c = T.tid; c < nc; c += T.nt) {
        const int md = E.cmode[c];
        if (md == BRK) continue;
        int before = 0;  // active contacts ahead of c in the unknowns
        for (int d = 0; d < c; ++d) before += E.cmode[d] == md;
        const int slot = 3 * (md == STK ? before : nstk + before);
        for (int a = 0; a < 3; ++a) {
            E.vctc[slot + a] = c;
            E.vcmp[slot + a] = a;
        }
        if (md == SLD) {
            const double s0 = E.dsig[3 * c], s1 = E.dsig[3 * c + 1];
            double ns = sqrt(s0 * s0 + s1 * s1);
            double u0, u1;
            if (ns > 1e-300) {
                u0 = s0 / ns;
                u1 = s1 / ns;
            } else {
                // no slip yet: hold the friction direction
                const double l0 = E.Ld[3 * c], l1 = E.Ld[3 * c + 1];
                const double nl = sqrt(l0 * l0 + l1 * l1);
                u0 = nl > 0 ? -l0 / nl : 1.0;
                u1 = nl > 0 ? -l1 / nl : 0.0;
                ns = 1e-300;
            }
            double* f = E.dfr + 4 * c;
            f[0] = u0;
            f[1] = u1;
            f[2] = double(E.mu[c]) * E.Ld[3 * c + 2] / ns;  // mu Lam_N / |sigma_T|
        }
    }
    if (T.tid == 0) {
        E.hdr[1] = m;
        E.hdr[2] = nstk;
    }
    // residual scales (largest free velocity, with the gravity step, and
    // largest impulse) as a team reduction
    double smax = 1e-300, lmax = 1e-300;
    for (int r = T.tid; r < k; r += T.nt) {
        const double a = fabs(E.gd[r]);
        smax = a > smax ? a : smax;
        const double l = fabs(E.Ld[r]);
        lmax = l > lmax ? l : lmax;
    }
    team_max2(T, E.redv, smax, lmax);  // its barrier also publishes the slots
    const double sg = P.dt * (fabs(P.gx) + fabs(P.gy) + fabs(P.gz));
    smax = smax > sg ? smax : sg;
    if (T.tid == 0) {
        E.dsc[4] = smax;
        E.dsc[5] = lmax;
    }
    for (int idx = T.tid; idx < m * m; idx += T.nt) {
        const int i = idx / m, j = idx - i * m;
        const int ci = E.vctc[i], ai = E.vcmp[i];
        const int cj = E.vctc[j], aj = E.vcmp[j];
        const int col = 3 * cj + aj;
        double v;
        if (E.cmode[ci] == SLD && ai < 2) {
            const double* f = E.dfr + 4 * ci;
            const double u0 = f[0], u1 = f[1], coef = f[2];
            const double h0 = (ai == 0) ? 1.0 - u0 * u0 : -u0 * u1;
            const double h1 = (ai == 0) ? -u0 * u1 : 1.0 - u1 * u1;
            v = coef * (h0 * E.Gd[(3 * ci) * k + col] + h1 * E.Gd[(3 * ci + 1) * k + col]);
            if (cj == ci && aj == ai) v += 1.0;
            if (cj == ci && aj == 2) v += double(E.mu[ci]) * (ai == 0 ? u0 : u1);
        } else {
            v = E.Gd[(3 * ci + ai) * k + col];
        }
        E.A[idx] = v;
    }
    // residual entries in parallel; their maximum and sum of squares by one
    // thread in index order
    for (int i = T.tid; i < m; i += T.nt) {
        const int c = E.vctc[i], a = E.vcmp[i];
        double f, rel;
        if (E.cmode[c] == SLD && a < 2) {
            const double* fr = E.dfr + 4 * c;
            f = E.Ld[3 * c + a] + double(E.mu[c]) * E.Ld[3 * c + 2] * fr[a];
            rel = fabs(f) / lmax;
        } else {
            f = E.dsig[3 * c + a];
            rel = fabs(f) / smax;
        }
        E.rhs[i] = -f;
        E.ytmp[i] = rel;
    }
    T.sync();
    if (T.tid == 0) {
        double res = 0, nrm = 0;
        for (int i = 0; i < m; ++i) {
            const double rel = E.ytmp[i];
            res = rel > res ? rel : res;
            nrm += rel * rel;
        }
        E.dsc[1] = res;
        E.dsc[3] = nrm;
    }
    T.sync();
}

// Newton refinement of the NCP solution (on Ld, FP64) with a fixed mode set,
// with active-set changes and backtracking.  When the equations are solved
// but an inequality of the mode set is violated, the offending contacts
// change mode (penetrating breaking contact -> sticking, negative normal
// impulse -> breaking, sticking impulse outside the cone -> sliding, slip not
// opposed by friction -> sticking) and the iteration continues; a step that
// increases the residual of the same mode set is halved once, then taken
// (longer backtracking spent evaluations without helping: more environments
// stalled than with the nearly plain Newton step).  Returns true on a
// consistent solution (also left in hdr[6]).  Run by wavefront 0 alone
// (T = wave_team of the environment's team): the iteration is a chain of
// small dependent steps whose team barriers cost more than the arithmetic.
template <class R, class TT>
DSIM_INLINE DSIM_HD bool polish(const TT& T, Env<R>& E, const Params& P) {
    const int k = E.k, nc = E.nc;
    const int max_changes = 2 * nc + 2;
    int changes = 0, since = 0;
    bool ok = false;
    if (T.tid == 0) {
        E.hdr[12] = 0;
        E.dsc[0] = 1e300;
    }
    T.sync();
    // bounded work: at most 4 (newton_iters + 1) evaluations per refinement;
    // a refinement that has not converged by then is rarely rescued by more
    // evaluations, and the next round restarts from more sweeps
    for (int guard = 0; guard < 4 * (P.newton_iters + 1); ++guard) {
        fp64_sigma(T, E);
        newton_system(T, E, P);
        const int m = E.hdr[1];
        if (T.tid == 0) {
            const double res = E.dsc[1], nrm = E.dsc[3];
            const int conv = (res <= P.ncp_tol) ? 1 : 0;
            int back = 0;
            if (!conv && since > 0 && nrm > E.dsc[0] && E.hdr[12] < 1) {
                back = 1;
                E.hdr[12] += 1;
                for (int r = 0; r < k; ++r) E.Ld[r] = 0.5 * (E.Ld1[r] + E.Ld[r]);
            } else {
                E.hdr[12] = 0;
                E.dsc[0] = nrm;
                for (int r = 0; r < k; ++r) E.Ld1[r] = E.Ld[r];
            }
            int viol = 0;
            // mode inequalities are checked at a solution of the mode
            // equations, or when Newton stalls on the current mode set
            if (conv || (!back && since >= P.newton_iters)) {
                const double smax = E.dsc[4], lmax = E.dsc[5];  // scales of this evaluation
                const double tl = 1e2 * P.ncp_tol;
                for (int c = 0; c < nc; ++c) {
                    const double L0 = E.Ld[3 * c], L1 = E.Ld[3 * c + 1], L2 = E.Ld[3 * c + 2];
                    const double S0 = E.dsig[3 * c], S1 = E.dsig[3 * c + 1], S2 = E.dsig[3 * c + 2];
                    const double mu = E.mu[c];
                    int md = E.cmode[c];
                    if (md == BRK) {
                        if (S2 < -tl * smax) md = STK;
                    } else if (L2 < -tl * lmax) {
                        md = BRK;
                    } else if (md == STK) {
                        if (sqrt(L0 * L0 + L1 * L1) > mu * L2 + tl * lmax) md = SLD;
                    } else if (L0 * S0 + L1 * S1 > 0) {
                        md = STK;
                    }
                    if (md != E.cmode[c]) {
                        ++viol;
                        E.cmode[c] = md;
                        if (md == BRK) E.Ld[3 * c] = E.Ld[3 * c + 1] = E.Ld[3 * c + 2] = 0;
                    }
                }
                if (viol) {
                    E.hdr[12] = 0;
                    E.dsc[0] = 1e300;
                }
            }
            E.hdr[9] = conv;
            E.hdr[11] = viol;
            E.hdr[13] = back;
        }
        T.sync();
        const int conv = E.hdr[9], viol = E.hdr[11];
        if (E.hdr[13]) continue;  // re-evaluate at the shortened step
        if (conv && !viol) {
            ok = true;
            break;
        }
        if (viol) {
            if (++changes > max_changes) break;
            since = 0;
            continue;
        }
        if (since >= P.newton_iters) break;
        ++since;
        factor_A(T, E, P.rank_tol);
        if (T.wave == 0) wave_lu_solve(T, E.A, m, E.hdr[4], E.rperm, E.cperm, E.rhs, E.ytmp, E.X);
        T.sync();
        for (int i = T.tid; i < m; i += T.nt) E.Ld[3 * E.vctc[i] + E.vcmp[i]] += E.X[i];
        T.sync();
    }
    if (ok && P.ncp_tol > 1e-9) {
        // A loose tolerance (the FP32 form's) stops the refinement one step
        // short of what FP64 Newton reaches on the converged mode set, and
        // the derivative inherits the solution's error through the reduced
        // system: take one more step (the system of the last evaluation is
        // current) and keep it when the residual decreases.
        const int m = E.hdr[1];
        const double res0 = E.dsc[1];
        for (int r = T.tid; r < k; r += T.nt) E.Ld1[r] = E.Ld[r];
        T.sync();
        factor_A(T, E, P.rank_tol);
        if (T.wave == 0) wave_lu_solve(T, E.A, m, E.hdr[4], E.rperm, E.cperm, E.rhs, E.ytmp, E.X);
        T.sync();
        for (int i = T.tid; i < m; i += T.nt) E.Ld[3 * E.vctc[i] + E.vcmp[i]] += E.X[i];
        T.sync();
        fp64_sigma(T, E);
        newton_system(T, E, P);
        if (!(E.dsc[1] < res0)) {
            for (int r = T.tid; r < k; r += T.nt) E.Ld[r] = E.Ld1[r];
            T.sync();
            fp64_sigma(T, E);
        }
    }
    if (T.tid == 0) E.hdr[6] = ok ? 1 : 0;
    T.sync();
    return ok;
}

// --------------------------------------------------------------------------
// damped semismooth Newton on the natural map (the fallback of the solve)
// --------------------------------------------------------------------------

// Projection of y onto the friction cone K_mu = {|x_T| <= mu x_N} and its
// Jacobian Pm (row-major 3x3): the identity inside the cone, zero in its
// polar cone, else the derivative of the boundary point
// beta (mu t, 1), beta = (mu |y_T| + y_N) / (mu^2 + 1), t = y_T / |y_T|.
DSIM_HD inline void cone_proj_jac(const double* y, double mu, double* p, double* Pm) {
    const double nt = sqrt(y[0] * y[0] + y[1] * y[1]);
    for (int i = 0; i < 9; ++i) Pm[i] = 0.0;
    if (nt <= mu * y[2]) {
        p[0] = y[0];
        p[1] = y[1];
        p[2] = y[2];
        Pm[0] = Pm[4] = Pm[8] = 1.0;
        return;
    }
    if (mu * nt <= -y[2]) {
        p[0] = p[1] = p[2] = 0.0;
        return;
    }
    const double c = 1.0 / (mu * mu + 1.0);
    const double beta = (mu * nt + y[2]) * c;
    const double t0 = y[0] / nt, t1 = y[1] / nt;
    const double db[3] = {c * mu * t0, c * mu * t1, c};
    const double h = mu * beta / nt;
    p[0] = mu * beta * t0;
    p[1] = mu * beta * t1;
    p[2] = beta;
    for (int j = 0; j < 3; ++j) {
        Pm[j] = mu * t0 * db[j];
        Pm[3 + j] = mu * t1 * db[j];
        Pm[6 + j] = db[j];
    }
    Pm[0] += h * (1.0 - t0 * t0);
    Pm[1] -= h * t0 * t1;
    Pm[3] -= h * t0 * t1;
    Pm[4] += h * (1.0 - t1 * t1);
}

// Sum and maximum over the wavefront (every lane gets the result; the host
// build's wavefront is one lane).
DSIM_HD inline double wave_sum(double a) {
#ifndef DSIM_HOST_BUILD
    for (int off = 32; off >= 1; off >>= 1) a += __shfl_xor(a, off, 64);
#endif
    return a;
}
DSIM_HD inline double wave_max(double a) {
#ifndef DSIM_HOST_BUILD
    for (int off = 32; off >= 1; off >>= 1) {
        const double o = __shfl_xor(a, off, 64);
        a = o > a ? o : a;
    }
#endif
    return a;
}

// The solve's fallback runs on wavefront 0 alone: its linear algebra is a
// chain of small dependent steps, and wavefront-level synchronisation keeps
// each step to a few LDS round trips (team barriers and per-step divisions
// made it an order of magnitude slower).  Lane r owns rows r, r + wsize, ...

// Natural map of the NCP at L (FP64): sigma = Gd L + gd (into dsig), per
// contact F_i = L_i - P_K(L_i - rho_i (sigma_i + Gamma(sigma_i))), Gamma the
// De Saxce term (0, 0, mu |sigma_T|), rho_i = 3 / trace(G_ii) as in the
// residual check.  With jac, also the blocks of its generalised Jacobian
//   dF_i/dL = [block i] (I - Pm_i) + C_i G_(i,:),  C_i = rho_i Pm_i D_i,
// D_i = I + e_N (mu u^T, 0), u = sigma_T / |sigma_T| (0 at no slip): Pm_i in
// pm, C_i in cm (9 per contact).  Leaves |F|^2, max_i |F_i| and max |L| in
// dsc[8], dsc[9], dsc[10].  Wavefront 0 only.
template <class R>
DSIM_INLINE DSIM_HD void wave_natural_map(const Team& T, Env<R>& E, const double* L, double* F, bool jac, double* pm,
                              double* cm) {
    const int k = E.k;
    for (int r = T.lane; r < k; r += T.wsize) {
        double s = E.gd[r];
        const double* g = E.Gd + r * k;
        for (int c = 0; c < k; ++c) s += g[c] * L[c];
        E.dsig[r] = s;
    }
    T.wave_sync();
    double a = 0, b = 0, l = 0;
    for (int c = T.lane; c < E.nc; c += T.wsize) {
        const double* sg = E.dsig + 3 * c;
        const double* Lc = L + 3 * c;
        const double mu = double(E.mu[c]);
        const double tr = E.Gd[(3 * c) * k + 3 * c] + E.Gd[(3 * c + 1) * k + 3 * c + 1] + E.Gd[(3 * c + 2) * k + 3 * c + 2];
        const double rho = tr > 0 ? 3.0 / tr : 1.0;
        const double st = sqrt(sg[0] * sg[0] + sg[1] * sg[1]);
        const double y[3] = {Lc[0] - rho * sg[0], Lc[1] - rho * sg[1], Lc[2] - rho * (sg[2] + mu * st)};
        double p[3], Pm[9];
        cone_proj_jac(y, mu, p, Pm);
        double n2 = 0;
        for (int i = 0; i < 3; ++i) {
            F[3 * c + i] = Lc[i] - p[i];
            n2 += F[3 * c + i] * F[3 * c + i];
            l = fabs(Lc[i]) > l ? fabs(Lc[i]) : l;
        }
        a += n2;
        b = sqrt(n2) > b ? sqrt(n2) : b;
        if (jac) {
            const double u0 = st > 0 ? sg[0] / st : 0.0, u1 = st > 0 ? sg[1] / st : 0.0;
            for (int i = 0; i < 3; ++i) {
                pm[9 * c + 3 * i] = Pm[3 * i];
                pm[9 * c + 3 * i + 1] = Pm[3 * i + 1];
                pm[9 * c + 3 * i + 2] = Pm[3 * i + 2];
                // (Pm D)_(i,:) = Pm_(i,:) + Pm_(i,2) (mu u0, mu u1, 0)
                cm[9 * c + 3 * i] = rho * (Pm[3 * i] + Pm[3 * i + 2] * mu * u0);
                cm[9 * c + 3 * i + 1] = rho * (Pm[3 * i + 1] + Pm[3 * i + 2] * mu * u1);
                cm[9 * c + 3 * i + 2] = rho * Pm[3 * i + 2];
            }
        }
    }
    a = wave_sum(a);
    b = wave_max(b);
    l = wave_max(l);
    if (T.lane == 0) {
        E.dsc[8] = a;
        E.dsc[9] = b;
        E.dsc[10] = l;
    }
    T.wave_sync();
}

// The natural map for the whole team (wavefront 0 computes; the results are
// in dsc[8..10] and F for every thread after the call).
template <class R>
DSIM_INLINE DSIM_HD void natural_map(const Team& T, Env<R>& E, const double* L, double* F, bool jac, double* pm, double* cm) {
    if (T.wave == 0) wave_natural_map(T, E, L, F, jac, pm, cm);
    T.sync();
}

// In-place Cholesky factor of the SPD k x k matrix M (row-major, lower
// triangle read): the strictly lower triangle gets L, dinv the reciprocals
// of L's diagonal.  Right-looking, the column scaling and the trailing
// update spread over the team (independent chains side by side; on one
// wavefront each lane's chain of dependent LDS updates was slower).
// Returns false (to every thread) on a pivot that is not positive.
DSIM_HD inline bool team_cholesky(const Team& T, double* M, double* dinv, int k) {
    for (int p = 0; p < k; ++p) {
        const double d = M[p * k + p];
        if (!(d > 0.0)) return false;
        const double inv = 1.0 / sqrt(d);
        for (int r = p + 1 + T.tid; r < k; r += T.nt) M[r * k + p] *= inv;
        if (T.tid == 0) dinv[p] = inv;
        T.sync();
        const int rem = k - p - 1;
        for (int idx = T.tid; idx < rem * rem; idx += T.nt) {
            const int i = p + 1 + idx / rem, j = p + 1 + idx % rem;
            if (j <= i) M[i * k + j] -= M[i * k + p] * M[j * k + p];
        }
        T.sync();
    }
    return true;
}

// Solves (L L^T) x = b with the factor of team_cholesky, x overwriting b.
// On the GPU lane r keeps x_r in a register and each step broadcasts the
// finished component with a cross-lane shuffle (k <= 64); the host build
// runs the same substitution serially.  Wavefront 0 only.
DSIM_HD inline void wave_cholesky_solve(const Team& T, const double* M, const double* dinv, int k, double* x) {
#ifdef DSIM_HOST_BUILD
    for (int i = 0; i < k; ++i) {
        double s = x[i];
        for (int j = 0; j < i; ++j) s -= M[i * k + j] * x[j];
        x[i] = s * dinv[i];
    }
    for (int i = k - 1; i >= 0; --i) {
        double s = x[i];
        for (int j = i + 1; j < k; ++j) s -= M[j * k + i] * x[j];
        x[i] = s * dinv[i];
    }
#else
    const int r = T.lane;
    double xr = r < k ? x[r] : 0.0;
    for (int i = 0; i < k; ++i) {
        const double xi = __shfl(xr, i, 64) * dinv[i];
        const double m = r > i && r < k ? M[r * k + i] : 0.0;
        xr = r == i ? xi : xr - m * xi;
    }
    for (int i = k - 1; i >= 0; --i) {
        const double xi = __shfl(xr, i, 64) * dinv[i];
        const double m = r < i ? M[i * k + r] : 0.0;
        xr = r == i ? xi : xr - m * xi;
    }
    if (r < k) x[r] = xr;
    T.wave_sync();
#endif
}

// Levenberg-Marquardt on the natural map F (a damped semismooth Newton
// method; Section II.B leaves the solver free), from the impulses in Ld:
// each iteration solves (H + lam (diag H + eps tr H / k)) d = -J^T F with
// H = J^T J (J the generalised Jacobian of natural_map, in FP64) and takes
// d when |F| decreases, else raises the damping.  It needs no mode set and
// the singular J of redundant contacts does not stop it.  Iterates until
// max_i |F_i| <= tol max |L|, the iteration cap or a stall (no 10% gain in
// 6 iterations) within `accept`; returns whether the residual ends within
// `accept` (near a kink of the natural map, at a contact close to a mode
// switch, the residual can stall above `tol`).  Uses A (J^T J), A2 (J, then
// the factor), rhs (F), ytmp (trial F), X (the step), Ld1 (trial), vrow /
// vcol (per-contact blocks), vdiag (-J^T F), dfr.  The products and the
// factorisation run on the team, the substitutions and the natural map on
// wavefront 0 (each phase on the layout measured fastest).
template <class R>
DSIM_HD bool lm_solve(const Team& T, Env<R>& E, double tol, double accept, int max_it) {
    const int k = E.k;
    double* H = E.A;
    double* Jm = E.A2;
    double* F = E.rhs;
    double* Ft = E.ytmp;
    double* d = E.X;
    double* Lt = E.Ld1;
    double* pm = E.vrow;
    double* cm = E.vcol;
    double damp = 1e-3, best = 1e300;
    int solves = 0, since = 0;
    bool stop = false;
    for (int it = 0; it < max_it && !stop; ++it) {
        if (T.tid == 0) E.hdr[8] += 1;  // iterations executed
        natural_map(T, E, E.Ld, F, true, pm, cm);
        const double f2 = E.dsc[8], fmax = E.dsc[9], lmax = E.dsc[10];
        if (fmax <= tol * lmax) return true;
        if (!(f2 == f2)) return false;
        // a stall (no 10% gain in 6 iterations) within `accept` ends it
        const double rel = fmax / lmax;
        since = rel < 0.9 * best ? 0 : since + 1;
        best = rel < 0.9 * best ? rel : best;
        if (since >= 6 && rel <= accept) break;
        for (int idx = T.tid; idx < k * k; idx += T.nt) {
            const int r = idx / k, j = idx - r * k;
            const int c = r / 3, a = r - 3 * c;
            const double* C = cm + 9 * c + 3 * a;
            double v = C[0] * E.Gd[(3 * c) * k + j] + C[1] * E.Gd[(3 * c + 1) * k + j] + C[2] * E.Gd[(3 * c + 2) * k + j];
            const int jb = j - 3 * c;
            if (jb >= 0 && jb < 3) v += (jb == a ? 1.0 : 0.0) - pm[9 * c + 3 * a + jb];
            Jm[idx] = v;
        }
        T.sync();
        for (int idx = T.tid; idx < k * k; idx += T.nt) {
            const int i = idx / k, j = idx - i * k;
            if (j > i) continue;
            double s = 0;
            for (int r = 0; r < k; ++r) s += Jm[r * k + i] * Jm[r * k + j];
            H[i * k + j] = s;
        }
        for (int i = T.tid; i < k; i += T.nt) {
            double g = 0;
            for (int r = 0; r < k; ++r) g -= Jm[r * k + i] * F[r];
            E.vdiag[i] = g;  // -J^T F, kept for the retries
        }
        T.sync();
        double tr = 0;
        for (int i = 0; i < k; ++i) tr += H[i * k + i];
        bool accepted = false;
        while (!accepted) {
            if (damp > 1e12 || ++solves > 4 * max_it) {
                stop = true;  // the final evaluation at Ld decides
                break;
            }
            if (T.tid == 0) E.hdr[3] += 1;  // damped solves executed
            const double floor = 1e-12 * tr / k;
            for (int idx = T.tid; idx < k * k; idx += T.nt) {
                const int i = idx / k, j = idx - i * k;
                if (j <= i) Jm[idx] = H[idx] + (i == j ? damp * (H[idx] + floor) : 0.0);
            }
            for (int i = T.tid; i < k; i += T.nt) d[i] = E.vdiag[i];
            T.sync();
            if (!team_cholesky(T, Jm, E.dfr, k)) {
                damp *= 4;
                continue;
            }
            if (T.wave == 0) wave_cholesky_solve(T, Jm, E.dfr, k, d);
            T.sync();
            for (int r = T.tid; r < k; r += T.nt) Lt[r] = E.Ld[r] + d[r];
            T.sync();
            natural_map(T, E, Lt, Ft, false, pm, cm);
            if (E.dsc[8] < f2) {
                for (int r = T.tid; r < k; r += T.nt) E.Ld[r] = Lt[r];
                T.sync();
                damp = damp / 3 > 1e-12 ? damp / 3 : 1e-12;
                accepted = true;
            } else {
                damp *= 4;
            }
        }
    }
    // sigma (dsig) and the residual at Ld, whatever ended the loop
    natural_map(T, E, E.Ld, F, false, pm, cm);
    return E.dsc[9] <= accept * E.dsc[10];
}

// ADMM (Section II.B lists it among the NCP solvers) on the De Saxce form
// of the NCP, from Ld = 0: with s = Gamma(sigma) held at its latest value,
// the NCP is the optimality condition of the convex cone program
//   min 1/2 L^T G L + (g + s)^T L  subject to  L in K_mu (each contact),
// split as L = z: L = (G + rho I)^-1 (rho (z - u) - g - s), z = P_K(L + u),
// u += L - z, then s from sigma = G z + g.  rho = trace(G) / k.  Every
// `check` iterations the natural map at z is evaluated; ends with Ld = z at
// max_i |F_i| <= tol max |z| or after max_it iterations (returns whether it
// converged).  Uses A ((G + rho I)^-1), A2 (its factor), Ld1 (L), rhs (u),
// ytmp (s), X, vrow / vcol (scratch of the natural map), dfr.
template <class R>
DSIM_HD bool admm_solve(const Team& T, Env<R>& E, double tol, int max_it, int check) {
    const int k = E.k, nc = E.nc;
    double* Minv = E.A;
    double* Fm = E.A2;
    double* z = E.Ld;
    double* L = E.Ld1;
    double* u = E.rhs;
    double* sv = E.ytmp;
    double tr = 0;
    for (int i = 0; i < k; ++i) tr += E.Gd[i * k + i];
    const double rho = tr > 0 ? tr / k : 1.0;
    for (int idx = T.tid; idx < k * k; idx += T.nt) {
        const int i = idx / k, j = idx - i * k;
        Fm[idx] = E.Gd[idx] + (i == j ? rho : 0.0);
    }
    for (int r = T.tid; r < k; r += T.nt) {
        z[r] = 0;
        u[r] = 0;
        sv[r] = 0;
    }
    T.sync();
    if (!team_cholesky(T, Fm, E.dfr, k)) return false;
    // explicit inverse, one column per thread (forward and back substitution)
    for (int col = T.tid; col < k; col += T.nt) {
        for (int i = 0; i < k; ++i) {
            double x = (i == col) ? 1.0 : 0.0;
            for (int j = 0; j < i; ++j) x -= Fm[i * k + j] * Minv[j * k + col];
            Minv[i * k + col] = x * E.dfr[i];
        }
        for (int i = k - 1; i >= 0; --i) {
            double x = Minv[i * k + col];
            for (int j = i + 1; j < k; ++j) x -= Fm[j * k + i] * Minv[j * k + col];
            Minv[i * k + col] = x * E.dfr[i];
        }
    }
    T.sync();
    for (int it = 0; it < max_it; ++it) {
        if (T.tid == 0) E.hdr[15] += 1;  // iterations executed
        // L = Minv (rho (z - u) - g - s)
        for (int r = T.tid; r < k; r += T.nt) E.X[r] = rho * (z[r] - u[r]) - E.gd[r] - sv[r];
        T.sync();
        for (int r = T.tid; r < k; r += T.nt) {
            double a = 0;
            for (int c = 0; c < k; ++c) a += Minv[r * k + c] * E.X[c];
            L[r] = a;
        }
        T.sync();
        // z = P_K(L + u), u += L - z (per contact)
        for (int c = T.tid; c < nc; c += T.nt) {
            const double y[3] = {L[3 * c] + u[3 * c], L[3 * c + 1] + u[3 * c + 1], L[3 * c + 2] + u[3 * c + 2]};
            double p[3], Pm[9];
            cone_proj_jac(y, double(E.mu[c]), p, Pm);
            for (int a = 0; a < 3; ++a) {
                z[3 * c + a] = p[a];
                u[3 * c + a] += L[3 * c + a] - p[a];
            }
        }
        T.sync();
        if ((it + 1) % check == 0) {
            natural_map(T, E, z, E.X, false, E.vrow, E.vcol);
            if (E.dsc[9] <= tol * E.dsc[10]) return true;
            if (!(E.dsc[8] == E.dsc[8])) return false;
        } else {
            // sigma at z for the De Saxce term
            for (int r = T.tid; r < k; r += T.nt) {
                double a = E.gd[r];
                for (int c = 0; c < k; ++c) a += E.Gd[r * k + c] * z[c];
                E.dsig[r] = a;
            }
            T.sync();
        }
        for (int c = T.tid; c < nc; c += T.nt) {
            const double* sg = E.dsig + 3 * c;
            sv[3 * c] = 0;
            sv[3 * c + 1] = 0;
            sv[3 * c + 2] = double(E.mu[c]) * sqrt(sg[0] * sg[0] + sg[1] * sg[1]);
        }
        T.sync();
    }
    return false;
}

// Modes of the impulses in Ld (reading R5 of the mode split, with the
// thresholds of mode_eps): breaking if the normal impulse is at most
// eps s_Lam, else sticking if the slip is at most eps s_sig, else sliding.
template <class R>
DSIM_HD void classify_modes(const Team& T, Env<R>& E, const Params& P) {
    // sigma at Ld is in dsig (the last natural_map); scales as the residual check
    if (T.tid == 0) {
        double smax, lmax;
        scales(E, P, smax, lmax);
        double sl = 1e-300;
        for (int c = 0; c < E.nc; ++c) sl = E.Ld[3 * c + 2] > sl ? E.Ld[3 * c + 2] : sl;
        for (int c = 0; c < E.nc; ++c) {
            const double* s = E.dsig + 3 * c;
            const double st = sqrt(s[0] * s[0] + s[1] * s[1]);
            int md = SLD;
            if (E.Ld[3 * c + 2] <= P.mode_eps * sl)
                md = BRK;
            else if (st <= P.mode_eps * smax)
                md = STK;
            E.cmode[c] = md;
        }
    }
    T.sync();
}

// The fallback pass of the solve, for an environment the first pass left
// unsolved, from that pass's impulses (in Ld): damped Newton on the natural
// map; if that does not converge, ADMM from zero impulses and damped Newton
// from its result.  A solution within the tolerance takes the modes its
// refinement confirms, or else (a contact at a mode boundary) the modes of
// the classification.  Returns whether it found one.
template <class R>
DSIM_HD bool fallback_solve(const Team& T, Env<R>& E, const Params& P) {
    // FP64 iterations: both forms converge them well below the FP32 form's
    // tolerance, so that its solution is as accurate as a refined one
    const double tol = 0.25 * (P.ncp_tol < 1e-11 ? P.ncp_tol : 1e-11);
    const double accept = 0.25 * P.ncp_tol;
    bool found = lm_solve(T, E, tol, accept, kLmIters);
    if (!found) {
        admm_solve(T, E, 1e-7, kAdmmIters, 20);
        found = lm_solve(T, E, tol, accept, kLmIters);
    }
    if (!found) return false;
    const int k = E.k;
    for (int r = T.tid; r < k; r += T.nt) E.vdiag[r] = E.Ld[r];
    classify_modes(T, E, P);
    if (T.wave == 0) polish(wave_team(T), E, P);
    T.sync();
    bool ok = E.hdr[6] != 0;
    if (ok) {
        // the refinement solves the mode equations; its result is kept only
        // if it also meets the natural-map tolerance
        natural_map(T, E, E.Ld, E.rhs, false, E.vrow, E.vcol);
        ok = E.dsc[9] <= accept * E.dsc[10];
    }
    if (!ok) {
        for (int r = T.tid; r < k; r += T.nt) E.Ld[r] = E.vdiag[r];
        T.sync();
        fp64_sigma(T, E);
        classify_modes(T, E, P);
    }
    return true;
}

// The NCP.  First pass (P.pass == 0): sweeps in working precision and
// refinement in FP64, repeated in rounds until the refinement reaches a
// consistent solution that meets the natural-map tolerance.  Fallback pass
// (P.pass == 1, run only for the environments the first pass left
// unsolved): fallback_solve from the first pass's impulses `lam_start` (its
// output).  Then the paper's reduced system at the solution, factorised for
// the derivative.
template <class R>
DSIM_HD void solve_ncp(const Team& T, Env<R>& E, const Params& P, const R* lam_start) {
    const int k = E.k;
    bool ok = false;
    if (P.pass == 1 && k > 0) {
        for (int r = T.tid; r < k; r += T.nt) E.Ld[r] = double(lam_start[3 * E.c0 + r]);
        T.sync();
        ok = fallback_solve(T, E, P);
        if (!ok) {
            // keep the first pass's impulses, with the modes they classify to
            for (int r = T.tid; r < k; r += T.nt) E.Ld[r] = double(lam_start[3 * E.c0 + r]);
            T.sync();
            fp64_sigma(T, E);
            classify_modes(T, E, P);
        }
    }
    for (int r = T.tid; r < k; r += T.nt) {
        E.Lam[r] = 0;
        E.sig[r] = E.g[r];
    }
    for (int c = T.tid; c < E.nc; c += T.nt) E.lmode[c] = BRK;
    T.sync();
    for (int round = 0; P.pass == 0 && round < P.ncp_rounds && k > 0; ++round) {
        nsgs(T, E, P.ncp_sweeps);
        if (round > 0) {
            // A round whose sweeps end in the state (impulses, sigma, modes)
            // they ended in the round before repeats that round exactly, its
            // failed refinement included, and so would every later round: the
            // solve ends here with the result of running them all.  Compared
            // bit for bit, so a NaN or a zero of the other sign differs.
            if (T.tid == 0) {
                int same = 1;
                for (int r = 0; r < k; ++r)
                    same &= (same_bits(E.Lam[r], E.Lam0[r]) && same_bits(E.sig[r], E.sig0[r])) ? 1 : 0;
                for (int c = 0; c < E.nc; ++c) same &= (E.lmode[c] == E.lmode0[c]) ? 1 : 0;
                E.hdr[14] = same;
            }
            T.sync();
            if (E.hdr[14]) break;
        }
        for (int r = T.tid; r < k; r += T.nt) {
            E.Ld[r] = double(E.Lam[r]);
            E.Lam0[r] = E.Lam[r];
            E.sig0[r] = E.sig[r];
        }
        for (int c = T.tid; c < E.nc; c += T.nt) {
            E.cmode[c] = E.lmode[c];
            E.lmode0[c] = E.lmode[c];
        }
        T.sync();
        if (T.wave == 0) polish(wave_team(T), E, P);
        T.sync();
        ok = E.hdr[6] != 0;
        if (ok) {
            // the refinement solves the equations of its mode set; the
            // solution is taken when it also meets the natural-map
            // tolerance, the test of the final residual check
            natural_map(T, E, E.Ld, E.rhs, false, E.vrow, E.vcol);
            ok = E.dsc[9] <= P.ncp_tol * E.dsc[10];
        }
        if (ok) break;
    }
    if (P.pass == 0 && !ok && k > 0) {
        // keep the Gauss-Seidel iterate and its modes (the fallback pass
        // starts from these impulses)
        for (int r = T.tid; r < k; r += T.nt) E.Ld[r] = double(E.Lam[r]);
        for (int c = T.tid; c < E.nc; c += T.nt) E.cmode[c] = E.lmode[c];
        T.sync();
    }
    for (int r = T.tid; r < k; r += T.nt) E.Lam[r] = R(E.Ld[r]);
    T.sync();
    if (k > 0) {
        fp64_sigma(T, E);
        reduced_vars(T, E);
        build_A(T, E);
        if (T.wave == 0) factor_A(wave_team(T), E, P.rank_tol);
        T.sync();
    }
    if (T.tid == 0) {
        E.hdr[5] = (ok || k == 0) ? 0 : ST_POLISH;
        if (k == 0) {
            E.hdr[1] = 0;
            E.hdr[4] = 0;
        }
    }
    T.sync();
}

// FP64 natural-map residual (Section II.B) |Lam - P_K(Lam - rho (sigma +
// Gamma(sigma)))| with rho = 3 / trace(G_ii), relative to the impulse scale;
// mode margins; sets the status bits.
template <class R>
DSIM_HD void residual_and_flags(const Team& T, Env<R>& E, const Params& P) {
    if (T.tid == 0) {
        const int k = E.k;
        double smax, lmax;
        scales(E, P, smax, lmax);
        double res = 0;
        bool degen = false;
        for (int c = 0; c < E.nc; ++c) {
            double s[3], L[3];
            for (int a = 0; a < 3; ++a) {
                s[a] = E.dsig[3 * c + a];
                L[a] = E.Ld[3 * c + a];
            }
            const double mu = double(E.mu[c]);
            const double tr = E.Gd[(3 * c) * k + 3 * c] + E.Gd[(3 * c + 1) * k + 3 * c + 1] +
                              E.Gd[(3 * c + 2) * k + 3 * c + 2];
            const double rho = tr > 0 ? 3.0 / tr : 1.0;
            const double st = sqrt(s[0] * s[0] + s[1] * s[1]);
            const double y[3] = {L[0] - rho * s[0], L[1] - rho * s[1], L[2] - rho * (s[2] + mu * st)};
            const double yt = sqrt(y[0] * y[0] + y[1] * y[1]);
            double p[3];
            if (yt <= mu * y[2]) {
                p[0] = y[0];
                p[1] = y[1];
                p[2] = y[2];
            } else if (mu * yt <= -y[2]) {
                p[0] = p[1] = p[2] = 0;
            } else {
                const double beta = (mu * yt + y[2]) / (mu * mu + 1.0);
                p[0] = mu * beta * y[0] / yt;
                p[1] = mu * beta * y[1] / yt;
                p[2] = beta;
            }
            const double r = sqrt((L[0] - p[0]) * (L[0] - p[0]) + (L[1] - p[1]) * (L[1] - p[1]) +
                                  (L[2] - p[2]) * (L[2] - p[2]));
            res = r > res ? r : res;
            const double eps = P.mode_eps;
            const double lt = sqrt(L[0] * L[0] + L[1] * L[1]);
            const int md = E.cmode[c];
            if (md == BRK) degen = degen || (s[2] <= eps * smax);
            if (md == STK) degen = degen || (L[2] <= eps * lmax) || (mu * L[2] - lt <= eps * lmax);
            if (md == SLD) degen = degen || (L[2] <= eps * lmax) || (st <= eps * smax);
        }
        int st = E.hdr[5];
        if (k > 0 && res > P.ncp_tol * lmax) st |= ST_NCP;
        if (E.hdr[4] < E.hdr[1]) st |= ST_RANK;
        if (degen) st |= ST_DEGEN;
        E.hdr[5] = st;
    }
    T.sync();
}

}  // namespace dsim
