// dsim_pipeline.h -- the NCP solve, the step outputs and the derivative
// phases of one environment team (continues dsim_core.h).
#pragma once

#include "dsim_core.h"

namespace dsim {

// Newton refinement of the NCP solution with the modes in E.cmode fixed
// (Section III.B equations).  Unknowns are the reduced variables of the
// current mode set; the Jacobian of the mode equations in those variables is
// the reduced matrix A itself (eq. 10), so each iteration builds and
// factorises A at the current impulse.  The sliding residual is the
// misalignment u_perp . Lam_T of the friction impulse with the slip
// direction; after each update sliding impulses are put back on the cone
// boundary.  Returns true if converged with a consistent mode set; on return
// A holds the factorisation at the final impulse.
template <class R>
DSIM_HD bool polish(const Team& T, Env<R>& E, const Params& P) {
    const int k = E.k, nc = E.nc;
    bool converged = false;
    for (int it = 0; it <= P.newton_iters; ++it) {
        // sigma in FP64 from the (working-precision) G, g, Lam
        for (int r = T.tid; r < k; r += T.nt) {
            double s = double(E.g[r]);
            for (int c = 0; c < k; ++c) s += double(E.G[r * k + c]) * double(E.Lam[c]);
            E.dsig[r] = s;
            E.sig[r] = R(s);
        }
        T.sync();
        reduced_vars(T, E);
        build_A(T, E);
        const int m = E.hdr[1];
        // residual of the mode equations, and its size relative to the scales
        if (T.tid == 0) {
            double smax = 1e-300, lmax = 1e-300;
            for (int r = 0; r < k; ++r) {
                double a = fabs(double(E.g[r]));
                smax = a > smax ? a : smax;
                double l = fabs(double(E.Lam[r]));
                lmax = l > lmax ? l : lmax;
            }
            double grav = fabs(P.gz) + fabs(P.gx) + fabs(P.gy);
            double sg = P.dt * grav;
            smax = smax > sg ? smax : sg;
            double res = 0;
            for (int i = 0; i < m; ++i) {
                const int c = E.vctc[i];
                double f;
                double rel;
                if (E.vcmp[i] == 1 && E.cmode[c] == SLD) {
                    const R* fr = E.sfr + 8 * c;
                    f = double(E.vdiag[i]) * (-double(fr[1]) * double(E.Lam[3 * c]) + double(fr[0]) * double(E.Lam[3 * c + 1]));
                    rel = fabs(f) / lmax;
                } else {
                    const R* rv = E.vrow + 3 * i;
                    f = double(rv[0]) * E.dsig[3 * c] + double(rv[1]) * E.dsig[3 * c + 1] + double(rv[2]) * E.dsig[3 * c + 2];
                    rel = fabs(f) / smax;
                }
                E.rhs[i] = -f;
                res = rel > res ? rel : res;
            }
            E.hdr[9] = (res <= P.ncp_tol) ? 1 : 0;
        }
        T.sync();
        factor_A(T, E, P.rank_tol);
        if (E.hdr[9]) {
            converged = true;
            break;
        }
        if (it == P.newton_iters) break;
        if (T.tid == 0) lu_solve(E.A, m, E.hdr[4], E.rperm, E.cperm, E.rhs, 1, E.ytmp, E.X, 1);
        T.sync();
        // Lam += C X, sliding impulses back on the cone
        for (int c = T.tid; c < nc; c += T.nt) {
            if (E.cmode[c] == BRK) continue;
            double d[3] = {0, 0, 0};
            for (int i = 0; i < m; ++i) {
                if (E.vctc[i] != c) continue;
                const double x = E.X[i];
                d[0] += double(E.vcol[3 * i]) * x;
                d[1] += double(E.vcol[3 * i + 1]) * x;
                d[2] += double(E.vcol[3 * i + 2]) * x;
            }
            double L0 = double(E.Lam[3 * c]) + d[0];
            double L1 = double(E.Lam[3 * c + 1]) + d[1];
            double L2 = double(E.Lam[3 * c + 2]) + d[2];
            if (E.cmode[c] == SLD) {
                double nt = sqrt(L0 * L0 + L1 * L1);
                double target = double(E.mu[c]) * L2;
                if (nt > 0 && target > 0) {
                    L0 *= target / nt;
                    L1 *= target / nt;
                }
            }
            E.Lam[3 * c] = R(L0);
            E.Lam[3 * c + 1] = R(L1);
            E.Lam[3 * c + 2] = R(L2);
        }
        T.sync();
    }
    // consistency of the mode set at the final impulse
    if (T.tid == 0) {
        bool ok = converged;
        double lmax = 1e-300;
        for (int r = 0; r < k; ++r) {
            double l = fabs(double(E.Lam[r]));
            lmax = l > lmax ? l : lmax;
        }
        const double tl = 1e3 * P.ncp_tol;
        for (int c = 0; c < nc && ok; ++c) {
            const double L0 = E.Lam[3 * c], L1 = E.Lam[3 * c + 1], L2 = E.Lam[3 * c + 2];
            const double mu = E.mu[c];
            if (E.cmode[c] == STK) {
                ok = ok && (L2 >= -tl * lmax) && (sqrt(L0 * L0 + L1 * L1) <= mu * L2 + tl * lmax);
            } else if (E.cmode[c] == SLD) {
                ok = ok && (L2 > 0) && (-(E.dsig[3 * c] * L0 + E.dsig[3 * c + 1] * L1) > 0);
            }
        }
        E.hdr[6] = ok ? 1 : 0;
    }
    T.sync();
    // breaking contacts must separate; checked with sigma at the final impulse
    for (int r = T.tid; r < k; r += T.nt) {
        double s = double(E.g[r]);
        for (int c = 0; c < k; ++c) s += double(E.G[r * k + c]) * double(E.Lam[c]);
        E.dsig[r] = s;
        E.sig[r] = R(s);
    }
    T.sync();
    if (T.tid == 0) {
        double smax = 1e-300;
        for (int r = 0; r < k; ++r) {
            double a = fabs(double(E.g[r]));
            smax = a > smax ? a : smax;
        }
        bool ok = E.hdr[6] != 0;
        for (int c = 0; c < nc && ok; ++c)
            if (E.cmode[c] == BRK) ok = ok && (E.dsig[3 * c + 2] >= -1e3 * P.ncp_tol * smax);
        E.hdr[6] = ok ? 1 : 0;
    }
    T.sync();
    return E.hdr[6] != 0;
}

template <class R>
DSIM_HD void solve_ncp(const Team& T, Env<R>& E, const Params& P) {
    const int k = E.k;
    for (int r = T.tid; r < k; r += T.nt) {
        E.Lam[r] = 0;
        E.sig[r] = E.g[r];
    }
    for (int c = T.tid; c < E.nc; c += T.nt) E.lmode[c] = BRK;
    T.sync();
    bool ok = false;
    for (int round = 0; round < P.ncp_rounds && k > 0; ++round) {
        nsgs(T, E, P.ncp_sweeps);
        for (int r = T.tid; r < k; r += T.nt) E.Lam0[r] = E.Lam[r];
        for (int c = T.tid; c < E.nc; c += T.nt) E.cmode[c] = E.lmode[c];
        T.sync();
        ok = polish(T, E, P);
        if (ok) break;
        // keep iterating from the Gauss-Seidel iterate
        for (int r = T.tid; r < k; r += T.nt) E.Lam[r] = E.Lam0[r];
        T.sync();
        update_sigma(T, E);
    }
    if (!ok && k > 0) {
        // factorisation at the Gauss-Seidel iterate with its modes
        for (int c = T.tid; c < E.nc; c += T.nt) E.cmode[c] = E.lmode[c];
        T.sync();
        update_sigma(T, E);
        for (int r = T.tid; r < k; r += T.nt) E.dsig[r] = double(E.sig[r]);
        T.sync();
        reduced_vars(T, E);
        build_A(T, E);
        factor_A(T, E, P.rank_tol);
    }
    if (T.tid == 0) E.hdr[5] = (ok || k == 0) ? 0 : ST_POLISH;
    if (k == 0 && T.tid == 0) { E.hdr[1] = 0; E.hdr[4] = 0; }
    T.sync();
}

// FP64 natural-map residual (Section II.B) and mode margins; sets status bits.
template <class R>
DSIM_HD void residual_and_flags(const Team& T, Env<R>& E, const Params& P) {
    if (T.tid == 0) {
        const int k = E.k;
        double lmax = 1e-300, smax = 1e-300;
        for (int r = 0; r < k; ++r) {
            double l = fabs(double(E.Lam[r]));
            lmax = l > lmax ? l : lmax;
            double a = fabs(double(E.g[r]));
            smax = a > smax ? a : smax;
        }
        double grav = fabs(P.gz) + fabs(P.gx) + fabs(P.gy);
        smax = smax > P.dt * grav ? smax : P.dt * grav;
        double res = 0;
        bool degen = false;
        for (int c = 0; c < E.nc; ++c) {
            double s[3], L[3];
            for (int a = 0; a < 3; ++a) {
                double v = double(E.g[3 * c + a]);
                for (int j = 0; j < k; ++j) v += double(E.G[(3 * c + a) * k + j]) * double(E.Lam[j]);
                s[a] = v;
                L[a] = double(E.Lam[3 * c + a]);
            }
            const double mu = double(E.mu[c]);
            const double tr = double(E.G[(3 * c) * k + 3 * c]) + double(E.G[(3 * c + 1) * k + 3 * c + 1]) +
                              double(E.G[(3 * c + 2) * k + 3 * c + 2]);
            const double rho = tr > 0 ? 3.0 / tr : 1.0;
            const double st = sqrt(s[0] * s[0] + s[1] * s[1]);
            double y[3] = {L[0] - rho * s[0], L[1] - rho * s[1], L[2] - rho * (s[2] + mu * st)};
            // projection onto the cone K_mu
            const double yt = sqrt(y[0] * y[0] + y[1] * y[1]);
            double p[3];
            if (yt <= mu * y[2]) {
                p[0] = y[0]; p[1] = y[1]; p[2] = y[2];
            } else if (mu * yt <= -y[2]) {
                p[0] = p[1] = p[2] = 0;
            } else {
                const double beta = (mu * yt + y[2]) / (mu * mu + 1.0);
                p[0] = mu * beta * y[0] / yt;
                p[1] = mu * beta * y[1] / yt;
                p[2] = beta;
            }
            const double r = sqrt((L[0] - p[0]) * (L[0] - p[0]) + (L[1] - p[1]) * (L[1] - p[1]) + (L[2] - p[2]) * (L[2] - p[2]));
            res = r > res ? r : res;
            const double eps = P.mode_eps;
            const double lt = sqrt(L[0] * L[0] + L[1] * L[1]);
            const int md = E.cmode[c];
            if (md == BRK) degen = degen || (s[2] <= eps * smax);
            if (md == STK) degen = degen || (L[2] <= eps * lmax) || (mu * L[2] - lt <= eps * lmax);
            if (md == SLD) degen = degen || (L[2] <= eps * lmax) || (st <= eps * smax);
        }
        int st = E.hdr[5];
        if (res > P.ncp_tol * lmax && k > 0) st |= ST_NCP;
        if (E.hdr[4] < E.hdr[1]) st |= ST_RANK;
        if (degen) st |= ST_DEGEN;
        E.hdr[5] = st;
    }
    T.sync();
}

// The step: kinematics, dynamics, factorisation, contacts, NCP, v+.
template <class R>
DSIM_HD void step_forward(const Team& T, Env<R>& E, const BatchView<R>& B, const Params& P, const R* q) {
    kinematics(T, E, B, q);
    mass_matrix(T, E);
    rnea(T, E, P, (const R*)nullptr, R(0), E.bias);
    ltdl(T, E);
    // free motion a_f = M^-1 (tau - b), v_f = v + dt a_f
    for (int i = T.tid; i < E.nv; i += T.nt) E.af[i] = E.tau[i] - E.bias[i];
    T.sync();
    if (T.tid == 0) ltdl_solve(E, E.af, 1);
    T.sync();
    for (int i = T.tid; i < E.nv; i += T.nt) E.vf[i] = E.v[i] + R(P.dt) * E.af[i];
    T.sync();
    if (E.k > 0) {
        contact_jacobian(T, E);
        delassus(T, E, P);
    }
    solve_ncp(T, E, P);
    // v+ = v_f + M^-1 J^T Lam, and a+ = a_f + M^-1 J^T Lam / dt
    const int n = E.nv, k = E.k;
    for (int i = T.tid; i < n; i += T.nt) {
        R s = 0;
        for (int c = 0; c < k; ++c) s += E.KT[c * n + i] * E.Lam[c];
        E.vn[i] = E.vf[i] + s;
        E.ap[i] = E.af[i] + s / R(P.dt);
    }
    T.sync();
    residual_and_flags(T, E, P);
}

template <class R>
DSIM_HD void write_step(const Team& T, Env<R>& E, R* v_next, R* lam, int8_t* mode, int32_t* status) {
    bool bad = false;
    for (int i = T.tid; i < E.nv; i += T.nt) {
        v_next[E.d0 + i] = E.vn[i];
        if (!(E.vn[i] == E.vn[i]) || fabs(double(E.vn[i])) > 1e300) bad = true;
    }
    for (int r = T.tid; r < E.k; r += T.nt) lam[3 * E.c0 + r] = E.Lam[r];
    for (int c = T.tid; c < E.nc; c += T.nt) mode[E.c0 + c] = int8_t(E.cmode[c]);
    if (bad) E.hdr[10] = 1;
    T.sync();
    if (T.tid == 0) status[E.e] = E.hdr[5] | (E.hdr[10] ? ST_NONFINITE : 0);
}

// --------------------------------------------------------------------------
// derivative phases
// --------------------------------------------------------------------------

// Per body: B_b (6x6, column m = B_b e_m) with
//   B_b w = I_b (w x V_b) + w x* (I_b V_b) + V_b x* (I_b w),
// and X_b (6x3): the change of the contact forces of body b under a rotation
// w of the body (the force direction is fixed in the world while the point
// moves): X_b w = sum_c (x_c x (w x f_c), w x f_c) with f_c = Lam_c / dt.
// Then composites over subtrees.
template <class R>
DSIM_HD void composites(const Team& T, Env<R>& E, const Params& P) {
    for (int b = T.tid; b < E.nb; b += T.nt) {
        const R* I = E.Iw + 10 * b;
        const R* Vb = E.V + 6 * b;
        R IV[6];
        iapply(I, Vb, IV);
        R* Bm = E.Bc + 36 * b;
        for (int mm = 0; mm < 6; ++mm) {
            R e[6] = {0, 0, 0, 0, 0, 0};
            e[mm] = 1;
            R wxV[6], t1[6], t2[6], Ie[6], t3[6];
            mxm(e, Vb, wxV);
            iapply(I, wxV, t1);
            mxf(e, IV, t2);
            iapply(I, e, Ie);
            mxf(Vb, Ie, t3);
            for (int r = 0; r < 6; ++r) Bm[6 * r + mm] = t1[r] + t2[r] + t3[r];
        }
        R* X = E.Ec + 18 * b;
        for (int i = 0; i < 18; ++i) X[i] = 0;
    }
    T.sync();
    if (T.tid == 0) {
        const R inv = R(1) / R(P.dt);
        for (int c = 0; c < E.nc; ++c) {
            const int b = E.cbody[c];
            R f[3] = {E.Lam[3 * c] * inv, E.Lam[3 * c + 1] * inv, E.Lam[3 * c + 2] * inv};
            const R* x = E.xw + 3 * c;
            R* X = E.Ec + 18 * b;
            for (int mm = 0; mm < 3; ++mm) {
                R e[3] = {0, 0, 0};
                e[mm] = 1;
                R gg[3], xg[3];
                cross3(e, f, gg);
                cross3(x, gg, xg);
                for (int r = 0; r < 3; ++r) {
                    X[3 * r + mm] += xg[r];
                    X[3 * (r + 3) + mm] += gg[r];
                }
            }
        }
    }
    T.sync();
    for (int i = T.tid; i < 54; i += T.nt)
        for (int b = E.nb - 1; b > 0; --b) {
            const int par = E.parent[b];
            if (par < 0) continue;
            if (i < 36) E.Bc[36 * par + i] += E.Bc[36 * b + i];
            else E.Ec[18 * par + i - 36] += E.Ec[18 * b + i - 36];
        }
    T.sync();
}

// Partial derivatives of the generalised forces tau = ID(q, v, a+) - J^T Lam/dt
// in q (tangent perturbations) and v, column by column from the motion of the
// subtree of each joint: see the derivation notes in the kernel source.
template <class R>
DSIM_HD void id_partials(const Team& T, Env<R>& E, const Params& P) {
    const int n = E.nv;
    // per dof vectors
    for (int d = T.tid; d < n; d += T.nt) {
        const int b = E.dbody[d];
        const int par = E.parent[b];
        const R* Sd = E.S + 6 * d;
        // row side
        iapply(E.Ic + 10 * b, Sd, E.IcS + 6 * d);
        const R* Bm = E.Bc + 36 * b;
        const R* X = E.Ec + 18 * b;
        for (int c = 0; c < 6; ++c) {
            R s = 0;
            for (int r = 0; r < 6; ++r) s += Bm[6 * r + c] * Sd[r];
            E.BtS[6 * d + c] = s;
        }
        for (int c = 0; c < 3; ++c) {
            R s = 0;
            for (int r = 0; r < 6; ++r) s += X[3 * r + c] * Sd[r];
            E.EtS[3 * d + c] = s;
        }
        // column side: parent body velocity and acceleration
        R Vl[6], Al[6];
        if (par >= 0) {
            for (int c = 0; c < 6; ++c) { Vl[c] = E.V[6 * par + c]; Al[c] = E.Acc[6 * par + c]; }
        } else {
            for (int c = 0; c < 6; ++c) Vl[c] = 0;
            Al[0] = 0; Al[1] = 0; Al[2] = 0;
            Al[3] = R(-P.gx); Al[4] = R(-P.gy); Al[5] = R(-P.gz);
        }
        R w[6], a[6], t[6];
        mxm(Sd, Vl, t);
        for (int c = 0; c < 6; ++c) w[c] = -t[c];      // w_j = -S_j x V_parent
        mxm(Sd, Al, a);
        mxm(w, Vl, t);
        for (int c = 0; c < 6; ++c) a[c] = -a[c] - t[c];  // a_j = -S_j x A_parent - w_j x V_parent
        R cj[6];
        mxm(E.V + 6 * b, Sd, t);
        for (int c = 0; c < 6; ++c) cj[c] = w[c] + t[c];  // c_j = -S_j x V_parent + V_b x S_j
        for (int c = 0; c < 6; ++c) { E.aj[6 * d + c] = a[c]; E.wj[6 * d + c] = w[c]; E.cj[6 * d + c] = cj[c]; }
        // ancestor-side vectors
        R y[6], u[6];
        mxf(Sd, E.Fc + 6 * b, y);
        iapply(E.Ic + 10 * b, a, u);
        for (int c = 0; c < 6; ++c) y[c] += u[c];
        for (int r = 0; r < 6; ++r) {
            R s = 0, s2 = 0;
            for (int c = 0; c < 6; ++c) { s += Bm[6 * r + c] * w[c]; s2 += Bm[6 * r + c] * Sd[c]; }
            R s3 = X[3 * r] * Sd[0] + X[3 * r + 1] * Sd[1] + X[3 * r + 2] * Sd[2];
            y[r] += s + s3;
            u[r] = s2;
        }
        for (int c = 0; c < 6; ++c) E.Yq[6 * d + c] = y[c];
        iapply(E.Ic + 10 * b, cj, t);
        for (int c = 0; c < 6; ++c) E.Yv[6 * d + c] = u[c] + t[c];
    }
    T.sync();
    for (int idx = T.tid; idx < n * n; idx += T.nt) {
        const int kk = idx / n, j = idx - kk * n;
        const int bk = E.dbody[kk], bj = E.dbody[j];
        R dq = 0, dv = 0;
        if ((E.bmask[bk] >> j) & 1ull) {
            // joint j moves body(k): the row's subtree composites
            dq = dot6(E.IcS + 6 * kk, E.aj + 6 * j) + dot6(E.BtS + 6 * kk, E.wj + 6 * j) + dot3(E.EtS + 3 * kk, E.S + 6 * j);
            dv = dot6(E.BtS + 6 * kk, E.S + 6 * j) + dot6(E.IcS + 6 * kk, E.cj + 6 * j);
        } else if ((E.bmask[bj] >> kk) & 1ull) {
            dq = dot6(E.S + 6 * kk, E.Yq + 6 * j);
            dv = dot6(E.S + 6 * kk, E.Yv + 6 * j);
        }
        E.dTq[idx] = dq;
        E.dTv[idx] = dv;
    }
    T.sync();
}

// E = d(J(q) v+)/dq at fixed v+ (contact point velocities of the moving
// subtree), plus (1/dt) J_N in gap mode 1.
template <class R>
DSIM_HD void velocity_partials(const Team& T, Env<R>& E, const Params& P) {
    const int nlev = E.hdr[0];
    for (int L = 0; L < nlev; ++L) {
        const int s = E.lstart[L], n = E.lstart[L + 1] - s;
        for (int i = T.tid; i < n; i += T.nt) body_velocity(E, E.vn, E.Vp, E.lorder[s + i]);
        T.sync();
    }
    const int n = E.nv, k = E.k;
    for (int idx = T.tid; idx < k * n; idx += T.nt) {
        const int row = idx / n, j = idx - row * n;
        const int c = row / 3, r = row - 3 * c;
        const int b = E.cbody[c];
        R val = 0;
        if ((E.bmask[b] >> j) & 1ull) {
            const R* x = E.xw + 3 * c;
            const R* Sj = E.S + 6 * j;
            const int par = E.parent[E.dbody[j]];
            // point velocities of x from the body and from the joint's parent
            R ui[3], ul[3], wl[3] = {0, 0, 0};
            const R* Vi = E.Vp + 6 * b;
            cross3(Vi, x, ui);
            ui[0] += Vi[3]; ui[1] += Vi[4]; ui[2] += Vi[5];
            ul[0] = ul[1] = ul[2] = 0;
            if (par >= 0) {
                const R* Vl = E.Vp + 6 * par;
                cross3(Vl, x, ul);
                ul[0] += Vl[3]; ul[1] += Vl[4]; ul[2] += Vl[5];
                wl[0] = Vl[0]; wl[1] = Vl[1]; wl[2] = Vl[2];
            }
            R du[3] = {ui[0] - ul[0], ui[1] - ul[1], ui[2] - ul[2]};
            R dx[3];
            cross3(Sj, x, dx);
            dx[0] += Sj[3]; dx[1] += Sj[4]; dx[2] += Sj[5];
            R t1[3], t2[3];
            cross3(Sj, du, t1);
            cross3(wl, dx, t2);
            val = t1[r] + t2[r];
            if (P.gap_mode == 1 && r == 2) val += dx[2] / R(P.dt);
        }
        E.E[idx] = val;
    }
    T.sync();
}

// Z = A^-1 B (FP64, basic solution), one thread per column of B; B selects
// the equation rows of each reduced variable (its row vector).
template <class R>
DSIM_HD void reduced_solve(const Team& T, Env<R>& E) {
    const int m = E.hdr[1], k = E.k, rank = E.hdr[4];
    for (int rho = T.tid; rho < k; rho += T.nt) {
        double* y = E.Ysc + rho * m;
        double* z = E.Z + rho * m;  // column rho of Z, contiguous
        for (int i = 0; i < m; ++i) {
            const int vi = E.rperm[i];
            const int c = E.vctc[vi];
            const int a = rho - 3 * c;
            y[i] = (a >= 0 && a < 3) ? double(E.vrow[3 * vi + a]) : 0.0;
        }
        for (int i = 0; i < rank; ++i) {
            double s = y[i];
            for (int j = 0; j < i; ++j) s -= E.A[i * m + j] * y[j];
            y[i] = s;
        }
        for (int i = rank; i < m; ++i) y[i] = 0;
        for (int i = rank - 1; i >= 0; --i) {
            double s = y[i];
            for (int j = i + 1; j < rank; ++j) s -= E.A[i * m + j] * y[j];
            y[i] = s / E.A[i * m + i];
        }
        for (int i = 0; i < m; ++i) z[E.cperm[i]] = y[i];
    }
    T.sync();
}

// Full Jacobian (Appendix D, eq. total_derivation, impulse form):
//   D0 = [-dt M^-1 dtau/dq, I - dt M^-1 dtau/dv, dt M^-1]
//   dv+/dtheta = D0 + M^-1 J^T dLam,  dLam = -C A^-1 B (J D0 + [E, 0, 0])
// regrouped as  T = -K C Z (K = M^-1 J^T, Z = A^-1 B), P = I + T J,
// Q = P M^-1:  dv+/dq = -dt Q dtau/dq + T E,  dv+/dv = P - dt Q dtau/dv,
// dv+/dtau = dt Q.
template <class R>
DSIM_HD void jacobian(const Team& T, Env<R>& E, const BatchView<R>& B, const Params& P,
                      R* dvdq, R* dvdv, R* dvdtau) {
    const int n = E.nv, k = E.k;
    rnea(T, E, P, E.ap, R(1) / R(P.dt), (R*)nullptr);
    composites(T, E, P);
    id_partials(T, E, P);
    velocity_partials(T, E, P);
    // M^-1, one column per thread
    for (int idx = T.tid; idx < n * n; idx += T.nt) E.Minv[idx] = ((idx / n) == (idx % n)) ? R(1) : R(0);
    T.sync();
    for (int j = T.tid; j < n; j += T.nt) ltdl_solve(E, E.Minv + j * n, 1);
    T.sync();
    const int m = E.hdr[1];
    R* CZ = E.P;  // k x k, reused before P is formed
    if (m > 0) {
        reduced_solve(T, E);
        for (int idx = T.tid; idx < k * k; idx += T.nt) {
            const int row = idx / k, rho = idx - row * k;
            const int c = row / 3, a = row - 3 * c;
            double s = 0;
            for (int i = 0; i < m; ++i)
                if (E.vctc[i] == c) s += double(E.vcol[3 * i + a]) * E.Z[rho * m + i];
            CZ[idx] = R(s);
        }
        T.sync();
        for (int idx = T.tid; idx < n * k; idx += T.nt) {
            const int i = idx / k, rho = idx - i * k;
            R s = 0;
            for (int c = 0; c < k; ++c) s += E.KT[c * n + i] * CZ[c * k + rho];
            E.T[idx] = -s;
        }
    } else {
        for (int idx = T.tid; idx < n * k; idx += T.nt) E.T[idx] = 0;
    }
    T.sync();
    for (int idx = T.tid; idx < n * n; idx += T.nt) {
        const int i = idx / n, j = idx - i * n;
        R s = (i == j) ? R(1) : R(0);
        for (int r = 0; r < k; ++r) s += E.T[i * k + r] * E.J[r * n + j];
        E.P[idx] = s;
    }
    T.sync();
    for (int idx = T.tid; idx < n * n; idx += T.nt) {
        const int i = idx / n, j = idx - i * n;
        R s = 0;
        for (int l = 0; l < n; ++l) s += E.P[i * n + l] * E.Minv[l * n + j];
        E.Q[idx] = s;
    }
    T.sync();
    const R dt = R(P.dt);
    const int off = B.jac_off[E.e];
    for (int idx = T.tid; idx < n * n; idx += T.nt) {
        const int i = idx / n, j = idx - i * n;
        R sq = 0, sv = 0, se = 0;
        for (int l = 0; l < n; ++l) {
            const R ql = E.Q[i * n + l];
            sq += ql * E.dTq[l * n + j];
            sv += ql * E.dTv[l * n + j];
        }
        for (int r = 0; r < k; ++r) se += E.T[i * k + r] * E.E[r * n + j];
        dvdq[off + idx] = -dt * sq + se;
        dvdv[off + idx] = E.P[idx] - dt * sv;
        dvdtau[off + idx] = dt * E.Q[idx];
    }
    T.sync();
}

// Reverse mode: the transpose of the Jacobian above applied to gbar,
//   tg = T^T gbar = -B^T A^-T C^T (K^T gbar),  pg = P^T gbar = gbar + J^T tg,
//   qg = Q^T gbar = M^-1 pg,
//   g_tau = dt qg,  g_v = pg - dt dtau/dv^T qg,  g_q = -dt dtau/dq^T qg + E^T tg.
// The transposed solve uses the same basic-solution operator as the forward
// derivative (its exact transpose), so both agree for rank-deficient A.
template <class R>
DSIM_HD void vjp(const Team& T, Env<R>& E, const BatchView<R>& B, const Params& P, const R* gbar,
                 R* gq, R* gv, R* gtau) {
    const int n = E.nv, k = E.k, m = E.hdr[1], rank = E.hdr[4];
    rnea(T, E, P, E.ap, R(1) / R(P.dt), (R*)nullptr);
    composites(T, E, P);
    id_partials(T, E, P);
    velocity_partials(T, E, P);
    R* gb = E.bias;  // gbar (the bias vector is no longer needed)
    R* pg = E.af;    // P^T gbar, then M^-1 P^T gbar
    R* tg = E.Lam0;  // T^T gbar (k)
    for (int i = T.tid; i < n; i += T.nt) gb[i] = gbar[E.d0 + i];
    T.sync();
    if (T.tid == 0) {
        // s = K^T gbar (k), s' = C^T s (m), y = (A^b)^T s', tg = -B^T y
        double* sp = E.rhs;
        double* z = E.ytmp;
        double* y = E.X;
        for (int i = 0; i < m; ++i) {
            const int c = E.vctc[i];
            double s = 0;
            for (int a = 0; a < 3; ++a) {
                double ka = 0;
                for (int j = 0; j < n; ++j) ka += double(E.KT[(3 * c + a) * n + j]) * double(gb[j]);
                s += double(E.vcol[3 * i + a]) * ka;
            }
            sp[i] = s;
        }
        for (int j = 0; j < rank; ++j) {
            double s = sp[E.cperm[j]];
            for (int i = 0; i < j; ++i) s -= E.A[i * m + j] * z[i];
            z[j] = s / E.A[j * m + j];
        }
        for (int i = rank - 1; i >= 0; --i) {
            double s = z[i];
            for (int j = i + 1; j < rank; ++j) s -= E.A[j * m + i] * z[j];
            z[i] = s;
        }
        for (int i = 0; i < m; ++i) y[E.rperm[i]] = (i < rank) ? z[i] : 0.0;
        for (int r = 0; r < k; ++r) tg[r] = 0;
        for (int i = 0; i < m; ++i) {
            const int c = E.vctc[i];
            for (int a = 0; a < 3; ++a) tg[3 * c + a] -= R(double(E.vrow[3 * i + a]) * y[i]);
        }
    }
    T.sync();
    for (int j = T.tid; j < n; j += T.nt) {
        R s = gb[j];
        for (int r = 0; r < k; ++r) s += E.J[r * n + j] * tg[r];
        pg[j] = s;
        E.vn[j] = s;  // keep P^T gbar (v+ already written out)
    }
    T.sync();
    if (T.tid == 0) ltdl_solve(E, pg, 1);
    T.sync();
    const R dt = R(P.dt);
    for (int j = T.tid; j < n; j += T.nt) {
        R sq = 0, sv = 0, se = 0;
        for (int l = 0; l < n; ++l) {
            sq += E.dTq[l * n + j] * pg[l];
            sv += E.dTv[l * n + j] * pg[l];
        }
        for (int r = 0; r < k; ++r) se += E.E[r * n + j] * tg[r];
        gq[E.d0 + j] = -dt * sq + se;
        gv[E.d0 + j] = E.vn[j] - dt * sv;
        gtau[E.d0 + j] = dt * pg[j];
    }
    T.sync();
}

// Full pipeline of one environment.
template <class R>
DSIM_HD void run_env(const Team& T, Env<R>& E, const BatchView<R>& B, const Params& P, int entry, int e,
                     const R* q, const R* v, const R* tau, const R* gbar, R* v_next, R* lam, int8_t* mode,
                     int32_t* status, R* o1, R* o2, R* o3) {
    load_env(T, E, B, e, v, tau);
    step_forward(T, E, B, P, q);
    write_step(T, E, v_next, lam, mode, status);
    if (entry == ENTRY_JAC) jacobian(T, E, B, P, o1, o2, o3);
    if (entry == ENTRY_VJP) vjp(T, E, B, P, gbar, o1, o2, o3);
    T.sync();
}

}  // namespace dsim
