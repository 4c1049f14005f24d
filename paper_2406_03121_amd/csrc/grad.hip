// Analytic nuclear gradient of the closed-shell Hartree-Fock energy (the
// atomic forces the paper obtains by differentiating its energy, sections 1
// and 4):
//
//   dE/dR_X = sum_{mu nu} D_{mu nu} dH_{mu nu}/dR_X
//           + 1/2 sum_{mu nu la si} P_{mu nu la si} d(mu nu|la si)/dR_X
//           - sum_{mu nu} W_{mu nu} dS_{mu nu}/dR_X + dE_nuc/dR_X,
//
// D the converged density, F its Fock matrix, W = D F D / 2 (energy-weighted
// density; the orthonormality constraint's term), and the symmetrised
// two-particle density P = D_{mu nu} D_{la si} - (D_{mu la} D_{nu si} +
// D_{mu si} D_{nu la}) / 4.  Only basis functions on atom X (and, for the
// nuclear attraction, the operator 1/|r - R_X|) depend on R_X; D and F need
// no response because the SCF energy is stationary.
//
// Integral derivatives by the McMurchie-Davidson Hermite expansion, with no
// run-time tables: the derivative of a primitive x_A^i e^{-a x_A^2} with
// respect to A_x is 2a x_A^(i+1) e^{-a x_A^2} - i x_A^(i-1) e^{-a x_A^2}, so
// each derivative integral is a combination of Hermite coefficients one
// order higher on the differentiated centre:
//   E^{00}_0 = 1,  E^{i+1,j}_t = E^{ij}_{t-1}/(2p) + X_PA E^{ij}_t + (t+1) E^{ij}_{t+1}
//   (and the same in j with X_PB), overlap (pi/p)^{3/2} K_AB prod_k E^{i_k j_k}_0,
//   kinetic from d^2/dx^2 of the ket factor, nuclear attraction
//   -Z_C (2 pi / p) K_AB sum_tuv E_t E_u E_v R_tuv(p, P - C), and
//   (ab|cd) = 2 pi^{5/2} / (p q sqrt(p + q)) K_AB K_CD
//             sum_tuv E^{ab}_tuv sum_{tau nu phi} (-1)^{tau+nu+phi} E^{cd}_{tau nu phi}
//             R_{t+tau, u+nu, v+phi}(pq/(p+q), P - Q),
//   R^n_000 = (-2 alpha)^n F_n(alpha |PC|^2), R^n_{t+1,u,v} = t R^{n+1}_{t-1,u,v} + X R^{n+1}_{tuv}.
// The fourth centre of a quartet follows from translational invariance
// (d/dA + d/dB + d/dC + d/dD = 0), as does the operator term of the
// nuclear attraction (d/dC = -(d/dA + d/dB) for each nucleus C).
//
// One-electron part: one lane per ordered shell pair (a, b), derivatives
// with respect to a's centre only (the (b, a) lane supplies b's).  Two-
// electron part: one wave per unique Schwarz-surviving shell quartet (with
// its permutation multiplicity), its lanes over the quartet's primitive
// quartets, summed over the wave.  Both take every primitive (no primitive
// screening) and add into the gradient with FP64 atomics.  This path runs
// once per geometry; it is written for clarity of the Hermite algebra, with
// its intermediates in per-lane arrays, not for speed.
#include <algorithm>
#include <cmath>
#include <vector>

#include "linalg.hpp"
#include "mess_internal.hpp"

namespace mess {

int zero_async(double *p, int64_t n, hipStream_t s);

struct GShell {
    double x, y, z;
    int l, prim0, nprim, bf0, atom;
};

// Cartesian components of l <= 2 in the library's order and their scales
// (mixed d components carry sqrt(3) relative to the (l,0,0) coefficients).
__device__ __forceinline__ void comp_exps(int l, int c, int &ex, int &ey, int &ez, double &sc) {
    sc = 1.0;
    if (l == 0) {
        ex = ey = ez = 0;
    } else if (l == 1) {
        ex = c == 0;
        ey = c == 1;
        ez = c == 2;
    } else {
        constexpr int t[6][3] = {{2, 0, 0}, {1, 1, 0}, {1, 0, 1}, {0, 2, 0}, {0, 1, 1}, {0, 0, 2}};
        ex = t[c][0];
        ey = t[c][1];
        ez = t[c][2];
        if (c == 1 || c == 2 || c == 4) sc = kSqrt3;
    }
}

// 1-D Hermite coefficients E[(i (J+1) + j) T + t], i <= I, j <= J,
// t <= i + j (T = I + J + 1 entries per (i, j)); E^{00}_0 = 1.
__device__ void md_e(int I, int J, double o2p, double PA, double PB, double *E) {
    const int T = I + J + 1;
    for (int n = 0; n < (I + 1) * (J + 1) * T; ++n) E[n] = 0.0;
    E[0] = 1.0;
    for (int i = 0; i <= I; ++i)
        for (int j = 0; j <= J; ++j) {
            if (i == 0 && j == 0) continue;
            const bool up_i = i > 0;
            const double X = up_i ? PA : PB;
            const double *src = E + ((up_i ? (i - 1) * (J + 1) + j : i * (J + 1) + j - 1)) * T;
            double *dst = E + (i * (J + 1) + j) * T;
            const int smax = i + j - 1;  // source t range
            for (int t = 0; t <= i + j; ++t) {
                double v = 0.0;
                if (t >= 1 && t - 1 <= smax) v += o2p * src[t - 1];
                if (t <= smax) v += X * src[t];
                if (t + 1 <= smax) v += (t + 1) * src[t + 1];
                dst[t] = v;
            }
        }
}

__device__ __forceinline__ int hidx(int t, int u, int v) {
    const int s = t + u + v, k = u + v;
    return s * (s + 1) * (s + 2) / 6 + k * (k + 1) / 2 + v;
}

constexpr int kGMaxN = 9;                                        // highest Boys order: (dd|dd) + 1
constexpr int kGRSize = (kGMaxN + 1) * (kGMaxN + 2) * (kGMaxN + 3) / 6;  // 220

// F_0..F_N(T), N <= 15 - 1: Taylor sum of F_N about T_k = k/16 (as many
// terms as the 16-column table holds, at most 8), downward recurrence; the
// large-T form above 60.
__device__ void grad_boys(int N, double T, const double *__restrict__ tab, double *F) {
    if (T < kBoysTmax) {
        const int k = __double2int_rn(T * kBoysInvStep);
        const double md = static_cast<double>(k) * (1.0 / kBoysInvStep) - T;
        const double *row = tab + k * kBoysN + N;
        const int nt = min(8, kBoysN - N);
        double f = row[nt - 1];
        for (int i = nt - 2; i >= 0; --i) f = row[i] + md * f / (i + 1);
        F[N] = f;
        const double e = exp(-T);
        for (int n = N - 1; n >= 0; --n) F[n] = (2.0 * T * F[n + 1] + e) / (2 * n + 1);
    } else {
        F[0] = 0.5 * sqrt(M_PI / T);
        for (int n = 0; n < N; ++n) F[n + 1] = F[n] * (2 * n + 1) * 0.5 / T;
    }
}

// R_tuv (t + u + v <= N) into R (compact order hidx), tmp of the same size.
__device__ void md_r(int N, double alpha, double X, double Y, double Z, const double *F, double *R, double *tmp) {
    double *cur = (N % 2 == 0) ? R : tmp, *nxt = (N % 2 == 0) ? tmp : R;
    // level n = N: only R^N_000
    double m2a = 1.0;
    for (int n = 0; n < N; ++n) m2a *= -2.0 * alpha;
    cur[0] = m2a * F[N];
    for (int n = N - 1; n >= 0; --n) {
        // nxt <- level n from cur (level n + 1, t + u + v <= N - n - 1)
        m2a /= -2.0 * alpha;
        nxt[0] = m2a * F[n];
        for (int s = 1; s <= N - n; ++s)
            for (int t = s; t >= 0; --t)
                for (int u = s - t; u >= 0; --u) {
                    const int v = s - t - u;
                    double r;
                    if (t > 0) r = (t > 1 ? (t - 1) * cur[hidx(t - 2, u, v)] : 0.0) + X * cur[hidx(t - 1, u, v)];
                    else if (u > 0) r = (u > 1 ? (u - 1) * cur[hidx(t, u - 2, v)] : 0.0) + Y * cur[hidx(t, u - 1, v)];
                    else r = (v > 1 ? (v - 1) * cur[hidx(t, u, v - 2)] : 0.0) + Z * cur[hidx(t, u, v - 1)];
                    nxt[hidx(t, u, v)] = r;
                }
        double *sw = cur;
        cur = nxt;
        nxt = sw;
    }
    // cur holds level 0; by the parity choice above it is R
}

// ------------------------------------------------------------ one-electron

// grad[atom][k] += 2 sum_{mu in a, nu in b} [D (dT + dV) - W dS]_{d/dA_k},
// grad[C][k] -= 2 D dV^C_{d/dA_k} for every nucleus C.
__global__ void __launch_bounds__(64) k_grad_1e(int nsh, const GShell *__restrict__ sh, const double *__restrict__ alpha,
                                                const double *__restrict__ ct, int nat, const double *__restrict__ xyz,
                                                const double *__restrict__ Zc, const double *__restrict__ tab, int N,
                                                const double *__restrict__ D, const double *__restrict__ W,
                                                double *__restrict__ grad) {
    const int lane = blockIdx.x * blockDim.x + threadIdx.x;
    if (lane >= nsh * nsh) return;
    const GShell A = sh[lane / nsh], B = sh[lane % nsh];
    const int la = A.l, lb = B.l, I = la + 1, J = lb + 2;
    const double AB[3] = {A.x - B.x, A.y - B.y, A.z - B.z};
    const double Ac[3] = {A.x, A.y, A.z}, Bc[3] = {B.x, B.y, B.z};
    const int na = (la + 1) * (la + 2) / 2, nb = (lb + 1) * (lb + 2) / 2;
    double E[3][4 * 5 * 8];   // i <= 3, j <= 4, t <= 7
    double Fb[8], R[kGRSize], tmp[kGRSize];
    double gA[3] = {0.0, 0.0, 0.0};
    for (int pa = 0; pa < A.nprim; ++pa)
        for (int pb = 0; pb < B.nprim; ++pb) {
            const double a = alpha[A.prim0 + pa], b = alpha[B.prim0 + pb];
            const double p = a + b, o2p = 0.5 / p, mu = a * b / p;
            const double cc = ct[A.prim0 + pa] * ct[B.prim0 + pb];
            const double Kab = exp(-mu * (AB[0] * AB[0] + AB[1] * AB[1] + AB[2] * AB[2]));
            const double P[3] = {(a * A.x + b * B.x) / p, (a * A.y + b * B.y) / p, (a * A.z + b * B.z) / p};
            for (int k = 0; k < 3; ++k) md_e(I, J, o2p, P[k] - Ac[k], P[k] - Bc[k], E[k]);
            const int T = I + J + 1;
            auto e1 = [&](int k, int i, int j, int t) -> double {
                return (i < 0 || j < 0 || t > i + j) ? 0.0 : E[k][(i * (J + 1) + j) * T + t];
            };
            const double sq = sqrt(M_PI / p);
            // 1-D overlap and kinetic factors
            auto s1 = [&](int k, int i, int j) -> double { return e1(k, i, j, 0) * sq; };
            auto t1 = [&](int k, int i, int j) -> double {
                return -0.5 * ((j >= 2 ? j * (j - 1) * s1(k, i, j - 2) : 0.0) - 2.0 * b * (2 * j + 1) * s1(k, i, j) +
                               4.0 * b * b * s1(k, i, j + 2));
            };
            // derivative (with respect to A_k) of a 1-D factor f(i, j)
            auto dA = [&](auto f, int k, int i, int j) -> double {
                return 2.0 * a * f(k, i + 1, j) - (i > 0 ? i * f(k, i - 1, j) : 0.0);
            };
            for (int ca = 0; ca < na; ++ca) {
                int ia[3];
                double sca;
                comp_exps(la, ca, ia[0], ia[1], ia[2], sca);
                for (int cb = 0; cb < nb; ++cb) {
                    int ib[3];
                    double scb;
                    comp_exps(lb, cb, ib[0], ib[1], ib[2], scb);
                    const int64_t mn = (int64_t)(A.bf0 + ca) * N + B.bf0 + cb;
                    const double w = cc * sca * scb * Kab;
                    const double Dmn = D[mn] * w, Wmn = W[mn] * w;
                    double S[3], Tk[3], dS[3], dT[3];
                    for (int k = 0; k < 3; ++k) {
                        S[k] = s1(k, ia[k], ib[k]);
                        Tk[k] = t1(k, ia[k], ib[k]);
                        dS[k] = dA(s1, k, ia[k], ib[k]);
                        dT[k] = dA(t1, k, ia[k], ib[k]);
                    }
                    for (int k = 0; k < 3; ++k) {
                        const int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
                        const double dSk = dS[k] * S[k1] * S[k2];
                        const double dTk = dT[k] * S[k1] * S[k2] + dS[k] * (Tk[k1] * S[k2] + S[k1] * Tk[k2]);
                        gA[k] += 2.0 * (Dmn * dTk - Wmn * dSk);
                    }
                }
            }
            // nuclear attraction, nucleus by nucleus
            const int Nv = la + lb + 1;
            for (int c = 0; c < nat; ++c) {
                const double PC[3] = {P[0] - xyz[3 * c], P[1] - xyz[3 * c + 1], P[2] - xyz[3 * c + 2]};
                grad_boys(Nv, p * (PC[0] * PC[0] + PC[1] * PC[1] + PC[2] * PC[2]), tab, Fb);
                md_r(Nv, p, PC[0], PC[1], PC[2], Fb, R, tmp);
                const double vpref = -Zc[c] * 2.0 * M_PI / p * Kab * cc;
                double gC[3] = {0.0, 0.0, 0.0};
                for (int ca = 0; ca < na; ++ca) {
                    int ia[3];
                    double sca;
                    comp_exps(la, ca, ia[0], ia[1], ia[2], sca);
                    for (int cb = 0; cb < nb; ++cb) {
                        int ib[3];
                        double scb;
                        comp_exps(lb, cb, ib[0], ib[1], ib[2], scb);
                        const double Dmn = D[(int64_t)(A.bf0 + ca) * N + B.bf0 + cb] * sca * scb * vpref;
                        for (int k = 0; k < 3; ++k) {
                            int e[3] = {ia[0], ia[1], ia[2]};
                            // sum_tuv dA_k[E] E E R over t_k <= i_k + 1 + j_k
                            double acc = 0.0;
                            for (int t = 0; t <= e[0] + ib[0] + (k == 0); ++t)
                                for (int u = 0; u <= e[1] + ib[1] + (k == 1); ++u)
                                    for (int v = 0; v <= e[2] + ib[2] + (k == 2); ++v) {
                                        const int tt[3] = {t, u, v};
                                        double f = 1.0;
                                        for (int q = 0; q < 3; ++q)
                                            f *= q == k ? 2.0 * a * e1(q, e[q] + 1, ib[q], tt[q]) -
                                                              (e[q] > 0 ? e[q] * e1(q, e[q] - 1, ib[q], tt[q]) : 0.0)
                                                        : e1(q, e[q], ib[q], tt[q]);
                                        acc += f * R[hidx(t, u, v)];
                                    }
                            gC[k] += Dmn * acc;
                        }
                    }
                }
                for (int k = 0; k < 3; ++k) {
                    gA[k] += 2.0 * gC[k];
                    atomicAdd(&grad[3 * c + k], -2.0 * gC[k]);
                }
            }
        }
    for (int k = 0; k < 3; ++k) atomicAdd(&grad[3 * A.atom + k], gA[k]);
}

// ------------------------------------------------------------ two-electron

__global__ void __launch_bounds__(64) k_grad_2e(int64_t nq, const int4 *__restrict__ quartets,
                                                const GShell *__restrict__ sh, const double *__restrict__ alpha,
                                                const double *__restrict__ ct, const double *__restrict__ tab, int N,
                                                const double *__restrict__ D, double *__restrict__ grad) {
    const int lane = threadIdx.x;
    for (int64_t qi = blockIdx.x; qi < nq; qi += gridDim.x) {
    const int4 q = quartets[qi];
    const GShell S[4] = {sh[q.x], sh[q.y], sh[q.z], sh[q.w]};
    const double mult = (q.x == q.y ? 1.0 : 2.0) * (q.z == q.w ? 1.0 : 2.0) * ((q.x == q.z && q.y == q.w) ? 1.0 : 2.0);
    const int la = S[0].l, lb = S[1].l, lc = S[2].l, ld = S[3].l;
    const int n4[4] = {(la + 1) * (la + 2) / 2, (lb + 1) * (lb + 2) / 2, (lc + 1) * (lc + 2) / 2,
                       (ld + 1) * (ld + 2) / 2};
    const int Ib = la + 1, Jb = lb + 1, Ik = lc + 1, Jk = ld;
    const int Tb = Ib + Jb + 1, Tk = Ik + Jk + 1;
    const int Lab = la + lb, Ltot = la + lb + lc + ld + 1;
    double Eb[3][4 * 4 * 7], Ek[3][4 * 3 * 6];
    double Fb[kGMaxN + 1], R[kGRSize], tmp[kGRSize];
    double X[4][56];
    double g[9] = {};  // d/dA, d/dB, d/dC (x, y, z each)
    const double c[4][3] = {{S[0].x, S[0].y, S[0].z}, {S[1].x, S[1].y, S[1].z}, {S[2].x, S[2].y, S[2].z},
                            {S[3].x, S[3].y, S[3].z}};
    // lane k takes primitive quartets k, k + 64, ... of this shell quartet
    const int n1 = S[1].nprim, n2 = S[2].nprim, n3 = S[3].nprim;
    const int npq = S[0].nprim * n1 * n2 * n3;
    for (int kq = lane; kq < npq; kq += 64) {
            const int p3 = kq % n3, p2 = (kq / n3) % n2, p1 = (kq / (n3 * n2)) % n1, p0 = kq / (n3 * n2 * n1);
            const double a = alpha[S[0].prim0 + p0], b = alpha[S[1].prim0 + p1];
            const double p = a + b;
            double ab2 = 0.0, P[3];
            for (int k = 0; k < 3; ++k) {
                P[k] = (a * c[0][k] + b * c[1][k]) / p;
                ab2 += (c[0][k] - c[1][k]) * (c[0][k] - c[1][k]);
            }
            const double Kab = exp(-a * b / p * ab2);
            for (int k = 0; k < 3; ++k) md_e(Ib, Jb, 0.5 / p, P[k] - c[0][k], P[k] - c[1][k], Eb[k]);
            const double cab = ct[S[0].prim0 + p0] * ct[S[1].prim0 + p1];
            {
                    const double cx = alpha[S[2].prim0 + p2], d = alpha[S[3].prim0 + p3];
                    const double qq = cx + d;
                    double cd2 = 0.0, Q[3];
                    for (int k = 0; k < 3; ++k) {
                        Q[k] = (cx * c[2][k] + d * c[3][k]) / qq;
                        cd2 += (c[2][k] - c[3][k]) * (c[2][k] - c[3][k]);
                    }
                    const double Kcd = exp(-cx * d / qq * cd2);
                    for (int k = 0; k < 3; ++k) md_e(Ik, Jk, 0.5 / qq, Q[k] - c[2][k], Q[k] - c[3][k], Ek[k]);
                    const double al = p * qq / (p + qq);
                    const double PQ[3] = {P[0] - Q[0], P[1] - Q[1], P[2] - Q[2]};
                    grad_boys(Ltot, al * (PQ[0] * PQ[0] + PQ[1] * PQ[1] + PQ[2] * PQ[2]), tab, Fb);
                    md_r(Ltot, al, PQ[0], PQ[1], PQ[2], Fb, R, tmp);
                    const double pref = 2.0 * pow(M_PI, 2.5) / (p * qq * sqrt(p + qq)) * Kab * Kcd * cab *
                                        ct[S[2].prim0 + p2] * ct[S[3].prim0 + p3] * 0.5 * mult;
                    auto eb = [&](int k, int i, int j, int t) -> double {
                        return (i < 0 || j < 0 || t > i + j) ? 0.0 : Eb[k][(i * (Jb + 1) + j) * Tb + t];
                    };
                    auto ek = [&](int k, int i, int j, int t) -> double {
                        return (i < 0 || j < 0 || t > i + j) ? 0.0 : Ek[k][(i * (Jk + 1) + j) * Tk + t];
                    };
                    for (int cc = 0; cc < n4[2]; ++cc) {
                        int ic[3];
                        double scc;
                        comp_exps(lc, cc, ic[0], ic[1], ic[2], scc);
                        for (int dc = 0; dc < n4[3]; ++dc) {
                            int id[3];
                            double scd;
                            comp_exps(ld, dc, id[0], id[1], id[2], scd);
                            // X[typ][tuv] = sum (-1)^(tau+nu+phi) E^{cd,typ}_{tau nu phi} R_{t+tau,u+nu,v+phi};
                            // typ 0: no derivative (t+u+v <= Lab+1), 1..3: d/dC_{x,y,z} (t+u+v <= Lab)
                            for (int typ = 0; typ < 4; ++typ) {
                                const int smax = typ == 0 ? Lab + 1 : Lab;
                                for (int s = 0; s <= smax; ++s)
                                    for (int t = s; t >= 0; --t)
                                        for (int u = s - t; u >= 0; --u) {
                                            const int v = s - t - u;
                                            double acc = 0.0;
                                            const int dx = typ == 1, dy = typ == 2, dz = typ == 3;
                                            for (int ta = 0; ta <= ic[0] + id[0] + dx; ++ta)
                                                for (int nu = 0; nu <= ic[1] + id[1] + dy; ++nu)
                                                    for (int ph = 0; ph <= ic[2] + id[2] + dz; ++ph) {
                                                        const int tt[3] = {ta, nu, ph};
                                                        double f = ((ta + nu + ph) & 1) ? -1.0 : 1.0;
                                                        for (int k = 0; k < 3; ++k)
                                                            f *= (typ == k + 1)
                                                                     ? 2.0 * cx * ek(k, ic[k] + 1, id[k], tt[k]) -
                                                                           (ic[k] > 0 ? ic[k] * ek(k, ic[k] - 1, id[k], tt[k]) : 0.0)
                                                                     : ek(k, ic[k], id[k], tt[k]);
                                                        acc += f * R[hidx(t + ta, u + nu, v + ph)];
                                                    }
                                            X[typ][hidx(t, u, v)] = acc;
                                        }
                            }
                            const int lam = S[2].bf0 + cc, sig = S[3].bf0 + dc;
                            for (int ac = 0; ac < n4[0]; ++ac) {
                                int ia[3];
                                double sca;
                                comp_exps(la, ac, ia[0], ia[1], ia[2], sca);
                                const int m = S[0].bf0 + ac;
                                for (int bc = 0; bc < n4[1]; ++bc) {
                                    int ib[3];
                                    double scb;
                                    comp_exps(lb, bc, ib[0], ib[1], ib[2], scb);
                                    const int n = S[1].bf0 + bc;
                                    const double Pd = D[(int64_t)m * N + n] * D[(int64_t)lam * N + sig] -
                                                      0.25 * (D[(int64_t)m * N + lam] * D[(int64_t)n * N + sig] +
                                                              D[(int64_t)m * N + sig] * D[(int64_t)n * N + lam]);
                                    const double w = Pd * pref * sca * scb * scc * scd;
                                    if (w == 0.0) continue;
                                    // centre A (typ 0..2), B (3..5): bra derivative with X[0];
                                    // centre C: bra without derivative with X[1..3]
                                    for (int k = 0; k < 3; ++k) {
                                        double sA = 0.0, sB = 0.0, sC = 0.0;
                                        for (int t = 0; t <= ia[0] + ib[0] + (k == 0); ++t)
                                            for (int u = 0; u <= ia[1] + ib[1] + (k == 1); ++u)
                                                for (int v = 0; v <= ia[2] + ib[2] + (k == 2); ++v) {
                                                    const int tt[3] = {t, u, v};
                                                    double fa = 1.0, fb = 1.0, f0 = 1.0;
                                                    for (int qd = 0; qd < 3; ++qd) {
                                                        const double e0 = eb(qd, ia[qd], ib[qd], tt[qd]);
                                                        if (qd == k) {
                                                            fa *= 2.0 * a * eb(qd, ia[qd] + 1, ib[qd], tt[qd]) -
                                                                  (ia[qd] > 0 ? ia[qd] * eb(qd, ia[qd] - 1, ib[qd], tt[qd]) : 0.0);
                                                            fb *= 2.0 * b * eb(qd, ia[qd], ib[qd] + 1, tt[qd]) -
                                                                  (ib[qd] > 0 ? ib[qd] * eb(qd, ia[qd], ib[qd] - 1, tt[qd]) : 0.0);
                                                        } else {
                                                            fa *= e0;
                                                            fb *= e0;
                                                        }
                                                        f0 *= e0;
                                                    }
                                                    const int h = hidx(t, u, v);
                                                    sA += fa * X[0][h];
                                                    sB += fb * X[0][h];
                                                    if (t + u + v <= Lab) sC += f0 * X[1 + k][h];
                                                }
                                        g[k] += w * sA;
                                        g[3 + k] += w * sB;
                                        g[6 + k] += w * sC;
                                    }
                                }
                            }
                        }
                    }
                }
        }
    // sums over the wave's primitive quartets
    for (int k = 0; k < 9; ++k)
        for (int off = 32; off > 0; off >>= 1) g[k] += __shfl_xor(g[k], off, 64);
    if (lane == 0)
        for (int k = 0; k < 3; ++k) {
            atomicAdd(&grad[3 * S[0].atom + k], g[k]);
            atomicAdd(&grad[3 * S[1].atom + k], g[3 + k]);
            atomicAdd(&grad[3 * S[2].atom + k], g[6 + k]);
            atomicAdd(&grad[3 * S[3].atom + k], -(g[k] + g[3 + k] + g[6 + k]));
        }
    }
}

// dE_nuc/dR_A = -sum_B Z_A Z_B (R_A - R_B) / |R_A - R_B|^3, one thread per atom
__global__ void k_grad_nuc(int nat, const double *__restrict__ xyz, const double *__restrict__ Zc,
                           double *__restrict__ grad) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= nat) return;
    double g[3] = {0.0, 0.0, 0.0};
    for (int b = 0; b < nat; ++b) {
        if (b == a) continue;
        const double d[3] = {xyz[3 * a] - xyz[3 * b], xyz[3 * a + 1] - xyz[3 * b + 1], xyz[3 * a + 2] - xyz[3 * b + 2]};
        const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        const double f = Zc[a] * Zc[b] / (r2 * sqrt(r2));
        for (int k = 0; k < 3; ++k) g[k] -= f * d[k];
    }
    for (int k = 0; k < 3; ++k) atomicAdd(&grad[3 * a + k], g[k]);
}

}  // namespace mess

using namespace mess;

extern "C" int mess_hf_gradient(const mess_basis *basis, const double *D, const double *F, double schwarz_tol,
                                double *grad, mess_stream stream) {
    if (!basis || !D || !F || !grad) {
        set_error("mess_hf_gradient: NULL argument");
        return MESS_E_ARG;
    }
    auto *B = const_cast<mess_basis *>(basis);
    if (B->n_mol != 1) {
        set_error("mess_hf_gradient: a batch of %d molecules; the gradient is built for one molecule", B->n_mol);
        return MESS_E_UNSUPPORTED;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int N = B->nbf, nat = B->nat, nsh = B->nsh;
    const double tau = schwarz_tol > 0.0 ? schwarz_tol : 0.0;
    // unique shell quartets that pass the Schwarz test, as mess_eri_quartets lists them
    int64_t counts[kNumClasses] = {};
    MESS_TRY(mess_eri_quartets(basis, tau, counts, nullptr));
    int64_t nq = 0;
    for (int c = 0; c < kNumClasses; ++c) nq += counts[c];
    std::vector<int32_t> qh(4 * std::max<int64_t>(nq, 1));
    if (nq) MESS_TRY(mess_eri_quartets(basis, tau, nullptr, qh.data()));
    std::vector<GShell> hs(nsh);
    for (int i = 0; i < nsh; ++i) {
        const int at = B->sh_atom[i];
        hs[i] = GShell{B->xyz[3 * at], B->xyz[3 * at + 1], B->xyz[3 * at + 2], B->sh_l[i], B->sh_prim0[i],
                       B->sh_np[i],     B->sh_bf0[i],      at};
    }
    const size_t np = B->alpha.size();
    double *d_alpha = nullptr, *d_ct = nullptr, *d_W = nullptr, *d_T = nullptr, *d_g = nullptr;
    GShell *d_sh = nullptr;
    int4 *d_q = nullptr;
    int rc = MESS_OK;
    auto fail = [&](int code, const char *what) {
        if (rc == MESS_OK) {
            rc = code;
            set_error("mess_hf_gradient: %s", what);
        }
    };
    if (hipMalloc(&d_alpha, sizeof(double) * np) != hipSuccess || hipMalloc(&d_ct, sizeof(double) * np) != hipSuccess ||
        hipMalloc(&d_W, sizeof(double) * (size_t)N * N) != hipSuccess ||
        hipMalloc(&d_T, sizeof(double) * (size_t)N * N) != hipSuccess ||
        hipMalloc(&d_g, sizeof(double) * 3 * nat) != hipSuccess || hipMalloc(&d_sh, sizeof(GShell) * nsh) != hipSuccess ||
        hipMalloc(&d_q, sizeof(int4) * std::max<int64_t>(nq, 1)) != hipSuccess)
        fail(MESS_E_NOMEM, "device allocation failed");
    if (rc == MESS_OK &&
        (hipMemcpyAsync(d_alpha, B->alpha.data(), sizeof(double) * np, hipMemcpyHostToDevice, s) != hipSuccess ||
         hipMemcpyAsync(d_ct, B->ctilde.data(), sizeof(double) * np, hipMemcpyHostToDevice, s) != hipSuccess ||
         hipMemcpyAsync(d_sh, hs.data(), sizeof(GShell) * nsh, hipMemcpyHostToDevice, s) != hipSuccess ||
         (nq && hipMemcpyAsync(d_q, qh.data(), sizeof(int4) * nq, hipMemcpyHostToDevice, s) != hipSuccess)))
        fail(MESS_E_DEVICE, "copy to the device failed");
    if (rc == MESS_OK) {
        // W = D F D / 2
        int r = gemm(s, false, false, N, N, N, 1.0, D, N, F, N, 0.0, d_T, N);
        if (r == MESS_OK) r = gemm(s, false, false, N, N, N, 0.5, d_T, N, D, N, 0.0, d_W, N);
        if (r == MESS_OK) r = zero_async(d_g, 3 * nat, s);
        if (r != MESS_OK) fail(r, "energy-weighted density failed");
    }
    if (rc == MESS_OK) {
        hipLaunchKernelGGL(k_grad_1e, dim3((unsigned)((nsh * nsh + 63) / 64)), dim3(64), 0, s, nsh, d_sh, d_alpha, d_ct,
                           nat, B->d_xyz, B->d_Zd, B->d_boys, N, D, d_W, d_g);
        if (nq)
            hipLaunchKernelGGL(k_grad_2e, dim3((unsigned)std::min<int64_t>(nq, 1 << 20)), dim3(64), 0, s, nq, d_q, d_sh, d_alpha,
                               d_ct, B->d_boys, N, D, d_g);
        hipLaunchKernelGGL(k_grad_nuc, dim3((unsigned)((nat + 63) / 64)), dim3(64), 0, s, nat, B->d_xyz, B->d_Zd, d_g);
        if (hipGetLastError() != hipSuccess) fail(MESS_E_DEVICE, "kernel launch failed");
    }
    if (rc == MESS_OK && (hipMemcpyAsync(grad, d_g, sizeof(double) * 3 * nat, hipMemcpyDeviceToHost, s) != hipSuccess ||
                          hipStreamSynchronize(s) != hipSuccess))
        fail(MESS_E_DEVICE, "gradient kernels failed");
    hipStreamSynchronize(s);
    for (void *p : {(void *)d_alpha, (void *)d_ct, (void *)d_W, (void *)d_T, (void *)d_g, (void *)d_sh, (void *)d_q})
        hipFree(p);
    return rc;
}
