/*
 * Plain FP64 CPU oracle for Gaussian-basis Hartree-Fock integrals.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code with the HIP library.
 *
 * What it computes (paper section 3, "Electronic Structure Theory in a
 * Nutshell"):
 *   - LCAO atomic-orbital basis of contracted Cartesian Gaussians (eq. 1),
 *     each function normalised to unit self-overlap;
 *   - the overlap matrix S (eq. 3) and the other closed-form Gaussian
 *     integrals the Roothaan equation (eq. 2) needs: kinetic T, nuclear
 *     attraction V, four-centre electron repulsion (mu nu|lambda sigma);
 *   - Coulomb / exchange matrices J, K from a density matrix.
 * The paper only says these integrals have closed forms; the form used here
 * is the McMurchie-Davidson Hermite-Gaussian expansion, written out directly:
 *   E coefficients:  E^{00}_0 = exp(-mu X_AB^2),
 *                    E^{i+1,j}_t = E^{ij}_{t-1}/(2p) + X_PA E^{ij}_t + (t+1) E^{ij}_{t+1},
 *                    E^{i,j+1}_t = E^{ij}_{t-1}/(2p) + X_PB E^{ij}_t + (t+1) E^{ij}_{t+1};
 *   Hermite integrals R^n_{000} = (-2 a)^n F_n(a |R|^2),
 *                    R^n_{t+1,u,v} = t R^{n+1}_{t-1,u,v} + X R^{n+1}_{t,u,v} (same for u, v);
 *   ERI = 2 pi^{5/2} / (p q sqrt(p+q)) sum_{tuv} E^{ab}_{tuv}
 *                    sum_{tau nu phi} (-1)^{tau+nu+phi} E^{cd}_{tau nu phi} R_{t+tau,u+nu,v+phi}.
 * Boys function F_n(T) = int_0^1 t^{2n} exp(-T t^2) dt, evaluated by its
 * power series e^{-T} sum_k (2T)^k / ((2n+1)(2n+3)...(2n+2k+1)) for T <= 20
 * and by F_0 = sqrt(pi/T) erf(sqrt T)/2 plus the upward recurrence
 * F_{n+1} = ((2n+1) F_n - e^{-T}) / (2T) above.
 *
 * Conventions: Cartesian components of a shell of angular momentum l are
 * ordered lexicographically with x fastest-decreasing: for l=2 that is
 * xx, xy, xz, yy, yz, zz.  Matrices are row-major N x N, ERIs are
 * (i j | k l) with i slowest.  Units are bohr and hartree.
 */
#include <stdlib.h>
#include <tgmath.h>
#include <string.h>

/* Arithmetic type: double by default; the test-suite also builds the same
 * source with -DOR_REAL="long double" as an extended-precision arbiter of
 * rounding-level differences. */
#ifndef OR_REAL
#define OR_REAL double
#endif
typedef OR_REAL real;
#define OR_PI ((real)3.14159265358979323846264338327950288L)

#define OR_LMAX 2          /* s, p, d shells */
#define OR_EMAX 5          /* E tables: i <= l+2 (kinetic), j <= l+2 */
#define OR_TMAX 11
#define OR_RL 9            /* R tables up to L = 8 */

/* ------------------------------------------------------------------ Boys */

static void boys_r(int nmax, real T, real *F)
{
    if (T <= 20.0) {
        real eT = exp(-T);
        for (int n = 0; n <= nmax; ++n) {
            real term = 1.0 / (2.0 * n + 1.0), sum = term;
            for (int k = 1; k < 1000; ++k) {
                term *= 2.0 * T / (2.0 * n + 2.0 * k + 1.0);
                sum += term;
                if (term < 1e-18 * sum) break;
            }
            F[n] = eT * sum;
        }
    } else {
        real eT = exp(-T);
        F[0] = 0.5 * sqrt(OR_PI / T) * erf(sqrt(T));
        for (int n = 0; n < nmax; ++n)
            F[n + 1] = ((2.0 * n + 1.0) * F[n] - eT) / (2.0 * T);
    }
}

/* ----------------------------------------------------------------- basis */

static real dfact(int n) /* n!! for odd n >= -1 */
{
    real r = 1.0;
    for (int k = n; k > 1; k -= 2) r *= k;
    return r;
}

static int ncart(int l) { return (l + 1) * (l + 2) / 2; }

static void cart_components(int l, int comp[][3])
{
    int c = 0;
    for (int lx = l; lx >= 0; --lx)
        for (int ly = l - lx; ly >= 0; --ly) {
            comp[c][0] = lx; comp[c][1] = ly; comp[c][2] = l - lx - ly; ++c;
        }
}

typedef struct {
    int nat, nsh, nbf;
    const int *Z;
    const double *xyz;
    const int *sh_atom, *sh_l, *sh_np;
    int *sh_prim;            /* first primitive of each shell */
    int *sh_bf;              /* first basis function of each shell */
    const double *alpha;     /* exponents */
    real *d;               /* [prim][6]: full coefficient per component */
} obasis;

/* Coefficient of primitive p for Cartesian component (lx,ly,lz) such that
 * the contracted function integrates to one when squared. */
static void normalise_shell(const obasis *B, int s)
{
    int l = B->sh_l[s], np = B->sh_np[s], p0 = B->sh_prim[s];
    int comp[6][3];
    cart_components(l, comp);
    for (int c = 0; c < ncart(l); ++c) {
        int lx = comp[c][0], ly = comp[c][1], lz = comp[c][2];
        real nprim[32];
        for (int p = 0; p < np; ++p) {
            real a = B->alpha[p0 + p];
            nprim[p] = pow(2.0 * a / OR_PI, 0.75) * pow(4.0 * a, 0.5 * l)
                       / sqrt(dfact(2 * lx - 1) * dfact(2 * ly - 1) * dfact(2 * lz - 1));
        }
        /* self-overlap of the un-renormalised contraction */
        real ss = 0.0;
        for (int p = 0; p < np; ++p)
            for (int q = 0; q < np; ++q) {
                real g = B->alpha[p0 + p] + B->alpha[p0 + q];
                real ov = pow(OR_PI / g, 1.5)
                            * dfact(2 * lx - 1) / pow(2.0 * g, lx)
                            * dfact(2 * ly - 1) / pow(2.0 * g, ly)
                            * dfact(2 * lz - 1) / pow(2.0 * g, lz);
                ss += B->d[(p0 + p) * 6 + c] * B->d[(p0 + q) * 6 + c] * nprim[p] * nprim[q] * ov;
            }
        real nc = 1.0 / sqrt(ss);
        for (int p = 0; p < np; ++p) B->d[(p0 + p) * 6 + c] *= nprim[p] * nc;
    }
}

static int basis_build(obasis *B, int nat, const int *Z, const double *xyz, int nsh,
                       const int *sh_atom, const int *sh_l, const int *sh_np,
                       const double *exps, const double *coefs)
{
    B->nat = nat; B->nsh = nsh; B->Z = Z; B->xyz = xyz;
    B->sh_atom = sh_atom; B->sh_l = sh_l; B->sh_np = sh_np; B->alpha = exps;
    B->sh_prim = (int *)malloc(sizeof(int) * (nsh + 1));
    B->sh_bf = (int *)malloc(sizeof(int) * (nsh + 1));
    int np = 0, nbf = 0;
    for (int s = 0; s < nsh; ++s) {
        if (sh_l[s] < 0 || sh_l[s] > OR_LMAX || sh_np[s] < 1 || sh_np[s] > 32) return -1;
        B->sh_prim[s] = np; B->sh_bf[s] = nbf;
        np += sh_np[s]; nbf += ncart(sh_l[s]);
    }
    B->sh_prim[nsh] = np; B->sh_bf[nsh] = nbf; B->nbf = nbf;
    B->d = (real *)malloc(sizeof(real) * 6 * (np > 0 ? np : 1));
    for (int p = 0; p < np; ++p)
        for (int c = 0; c < 6; ++c) B->d[p * 6 + c] = coefs[p];
    for (int s = 0; s < nsh; ++s) normalise_shell(B, s);
    return 0;
}

static void basis_free(obasis *B)
{
    free(B->sh_prim); free(B->sh_bf); free(B->d);
}

static const double *centre(const obasis *B, int s) { return B->xyz + 3 * B->sh_atom[s]; }

/* ------------------------------------------------------- Hermite tables */

typedef real Etab[OR_EMAX][OR_EMAX][OR_TMAX];

/* One Cartesian direction; a on A, b on B, Xab = A - B. */
static void hermite_E(int imax, int jmax, real a, real b, real Xab, Etab E)
{
    real p = a + b, mu = a * b / p;
    real Xpa = -b / p * Xab, Xpb = a / p * Xab;
    memset(E, 0, sizeof(Etab));
    E[0][0][0] = exp(-mu * Xab * Xab);
    for (int i = 0; i <= imax; ++i)
        for (int j = 0; j <= jmax; ++j) {
            if (i == 0 && j == 0) continue;
            for (int t = 0; t <= i + j; ++t) {
                real lo, mid, hi, shift;
                if (j == 0) {
                    lo = t > 0 ? E[i - 1][0][t - 1] : 0.0;
                    mid = E[i - 1][0][t];
                    hi = E[i - 1][0][t + 1];
                    shift = Xpa;
                } else {
                    lo = t > 0 ? E[i][j - 1][t - 1] : 0.0;
                    mid = E[i][j - 1][t];
                    hi = E[i][j - 1][t + 1];
                    shift = Xpb;
                }
                E[i][j][t] = lo / (2.0 * p) + shift * mid + (t + 1) * hi;
            }
        }
}

typedef real Rtab[OR_RL][OR_RL][OR_RL][OR_RL];   /* [n][t][u][v] */

static void hermite_R(int L, real a, real X, real Y, real Zc, Rtab R)
{
    real T = a * (X * X + Y * Y + Zc * Zc);
    real F[OR_RL + 1];
    boys_r(L, T, F);
    real f = 1.0;
    for (int n = 0; n <= L; ++n) {
        R[n][0][0][0] = f * F[n];
        f *= -2.0 * a;
    }
    for (int n = L - 1; n >= 0; --n)
        for (int t = 0; t <= L - n; ++t)
            for (int u = 0; u <= L - n - t; ++u)
                for (int v = 0; v <= L - n - t - u; ++v) {
                    if (t + u + v == 0) continue;
                    real val;
                    if (t > 0)
                        val = (t > 1 ? (t - 1) * R[n + 1][t - 2][u][v] : 0.0) + X * R[n + 1][t - 1][u][v];
                    else if (u > 0)
                        val = (u > 1 ? (u - 1) * R[n + 1][t][u - 2][v] : 0.0) + Y * R[n + 1][t][u - 1][v];
                    else
                        val = (v > 1 ? (v - 1) * R[n + 1][t][u][v - 2] : 0.0) + Zc * R[n + 1][t][u][v - 1];
                    R[n][t][u][v] = val;
                }
}

/* ------------------------------------------------------ one-electron */

/* S, T, V block of shells (sa, sb): out arrays [na*nb] row-major. */
static void one_electron_block(const obasis *B, int sa, int sb, real *S, real *Tk, real *V)
{
    int la = B->sh_l[sa], lb = B->sh_l[sb];
    int na = ncart(la), nb = ncart(lb);
    int ca[6][3], cb[6][3];
    cart_components(la, ca); cart_components(lb, cb);
    const double *A = centre(B, sa), *Bc = centre(B, sb);
    for (int k = 0; k < na * nb; ++k) S[k] = Tk[k] = V[k] = 0.0;
    Etab *E = (Etab *)malloc(sizeof(Etab) * 3);
    Rtab *R = (Rtab *)malloc(sizeof(Rtab));
    for (int p = 0; p < B->sh_np[sa]; ++p)
        for (int q = 0; q < B->sh_np[sb]; ++q) {
            int ip = B->sh_prim[sa] + p, iq = B->sh_prim[sb] + q;
            real a = B->alpha[ip], b = B->alpha[iq], pp = a + b;
            real P[3];
            for (int x = 0; x < 3; ++x) {
                hermite_E(la, lb + 2, a, b, A[x] - Bc[x], E[x]);
                P[x] = (a * A[x] + b * Bc[x]) / pp;
            }
            real s1 = sqrt(OR_PI / pp);
            for (int i = 0; i < na; ++i)
                for (int j = 0; j < nb; ++j) {
                    real cc = B->d[ip * 6 + i] * B->d[iq * 6 + j];
                    real sd[3], td[3];
                    for (int x = 0; x < 3; ++x) {
                        int li = ca[i][x], lj = cb[j][x];
                        sd[x] = E[x][li][lj][0] * s1;
                        real tp2 = E[x][li][lj + 2][0] * s1;
                        real tm2 = lj >= 2 ? E[x][li][lj - 2][0] * s1 : 0.0;
                        td[x] = -2.0 * b * b * tp2 + b * (2 * lj + 1) * sd[x] - 0.5 * lj * (lj - 1) * tm2;
                    }
                    S[i * nb + j] += cc * sd[0] * sd[1] * sd[2];
                    Tk[i * nb + j] += cc * (td[0] * sd[1] * sd[2] + sd[0] * td[1] * sd[2] + sd[0] * sd[1] * td[2]);
                }
            for (int C = 0; C < B->nat; ++C) {
                const double *Cc = B->xyz + 3 * C;
                hermite_R(la + lb, pp, P[0] - Cc[0], P[1] - Cc[1], P[2] - Cc[2], *R);
                real pref = -B->Z[C] * 2.0 * OR_PI / pp;
                for (int i = 0; i < na; ++i)
                    for (int j = 0; j < nb; ++j) {
                        real cc = B->d[ip * 6 + i] * B->d[iq * 6 + j];
                        int lx = ca[i][0] + cb[j][0], ly = ca[i][1] + cb[j][1], lz = ca[i][2] + cb[j][2];
                        real sum = 0.0;
                        for (int t = 0; t <= lx; ++t)
                            for (int u = 0; u <= ly; ++u)
                                for (int v = 0; v <= lz; ++v)
                                    sum += E[0][ca[i][0]][cb[j][0]][t] * E[1][ca[i][1]][cb[j][1]][u]
                                           * E[2][ca[i][2]][cb[j][2]][v] * (*R)[0][t][u][v];
                        V[i * nb + j] += cc * pref * sum;
                    }
            }
        }
    free(E); free(R);
}

/* --------------------------------------------------------------- ERIs */

/* Contracted block (sa sb | sc sd), out[na*nb*nc*nd] with a slowest. */
static void eri_block(const obasis *B, int sa, int sb, int sc, int sd, real *out)
{
    int l[4] = {B->sh_l[sa], B->sh_l[sb], B->sh_l[sc], B->sh_l[sd]};
    int sh[4] = {sa, sb, sc, sd};
    int n[4], comp[4][6][3];
    for (int k = 0; k < 4; ++k) { n[k] = ncart(l[k]); cart_components(l[k], comp[k]); }
    int ntot = n[0] * n[1] * n[2] * n[3];
    for (int k = 0; k < ntot; ++k) out[k] = 0.0;
    const double *A = centre(B, sa), *Bc = centre(B, sb), *C = centre(B, sc), *D = centre(B, sd);
    Etab *Eab = (Etab *)malloc(sizeof(Etab) * 3);
    Etab *Ecd = (Etab *)malloc(sizeof(Etab) * 3);
    Rtab *R = (Rtab *)malloc(sizeof(Rtab));
    int L = l[0] + l[1] + l[2] + l[3];
    for (int pa = 0; pa < B->sh_np[sa]; ++pa)
    for (int pb = 0; pb < B->sh_np[sb]; ++pb) {
        int ia = B->sh_prim[sa] + pa, ib = B->sh_prim[sb] + pb;
        real a = B->alpha[ia], b = B->alpha[ib], p = a + b, P[3];
        for (int x = 0; x < 3; ++x) {
            hermite_E(l[0], l[1], a, b, A[x] - Bc[x], Eab[x]);
            P[x] = (a * A[x] + b * Bc[x]) / p;
        }
        for (int pc = 0; pc < B->sh_np[sc]; ++pc)
        for (int pd = 0; pd < B->sh_np[sd]; ++pd) {
            int ic = B->sh_prim[sc] + pc, id = B->sh_prim[sd] + pd;
            real c = B->alpha[ic], d = B->alpha[id], q = c + d, Q[3];
            for (int x = 0; x < 3; ++x) {
                hermite_E(l[2], l[3], c, d, C[x] - D[x], Ecd[x]);
                Q[x] = (c * C[x] + d * D[x]) / q;
            }
            real rho = p * q / (p + q);
            hermite_R(L, rho, P[0] - Q[0], P[1] - Q[1], P[2] - Q[2], *R);
            real pref = 2.0 * pow(OR_PI, 2.5) / (p * q * sqrt(p + q));
            int k = 0;
            for (int i = 0; i < n[0]; ++i)
            for (int j = 0; j < n[1]; ++j)
            for (int kk = 0; kk < n[2]; ++kk)
            for (int ll = 0; ll < n[3]; ++ll, ++k) {
                const int *ci = comp[0][i], *cj = comp[1][j], *ck = comp[2][kk], *cl = comp[3][ll];
                real sum = 0.0;
                for (int t = 0; t <= ci[0] + cj[0]; ++t)
                for (int u = 0; u <= ci[1] + cj[1]; ++u)
                for (int v = 0; v <= ci[2] + cj[2]; ++v) {
                    real eb = Eab[0][ci[0]][cj[0]][t] * Eab[1][ci[1]][cj[1]][u] * Eab[2][ci[2]][cj[2]][v];
                    real inner = 0.0;
                    for (int tau = 0; tau <= ck[0] + cl[0]; ++tau)
                    for (int nu = 0; nu <= ck[1] + cl[1]; ++nu)
                    for (int phi = 0; phi <= ck[2] + cl[2]; ++phi) {
                        real ek = Ecd[0][ck[0]][cl[0]][tau] * Ecd[1][ck[1]][cl[1]][nu] * Ecd[2][ck[2]][cl[2]][phi];
                        real sgn = ((tau + nu + phi) & 1) ? -1.0 : 1.0;
                        inner += sgn * ek * (*R)[0][t + tau][u + nu][v + phi];
                    }
                    sum += eb * inner;
                }
                real cc = B->d[ia * 6 + i] * B->d[ib * 6 + j] * B->d[ic * 6 + kk] * B->d[id * 6 + ll];
                out[k] += cc * pref * sum;
            }
        }
    }
    free(Eab); free(Ecd); free(R);
    (void)sh;
}

void oracle_boys(int nmax, double T, double *F)
{
    real Fr[64];
    boys_r(nmax, (real)T, Fr);
    for (int n = 0; n <= nmax; ++n) F[n] = (double)Fr[n];
}

/* ------------------------------------------------------------ exports */

#define MOL_ARGS int nat, const int *Z, const double *xyz, int nsh, const int *sh_atom, \
                 const int *sh_l, const int *sh_np, const double *exps, const double *coefs
#define MOL_PASS nat, Z, xyz, nsh, sh_atom, sh_l, sh_np, exps, coefs

int oracle_nbf(int nsh, const int *sh_l)
{
    int n = 0;
    for (int s = 0; s < nsh; ++s) n += ncart(sh_l[s]);
    return n;
}

double oracle_nuclear_repulsion(int nat, const int *Z, const double *xyz)
{
    double e = 0.0;
    for (int a = 0; a < nat; ++a)
        for (int b = 0; b < a; ++b) {
            double dx = xyz[3 * a] - xyz[3 * b], dy = xyz[3 * a + 1] - xyz[3 * b + 1],
                   dz = xyz[3 * a + 2] - xyz[3 * b + 2];
            e += Z[a] * Z[b] / sqrt(dx * dx + dy * dy + dz * dz);
        }
    return e;
}

/* Normalised primitive coefficients, [sum nprim][6] (component-resolved). */
int oracle_coefficients(MOL_ARGS, double *out)
{
    obasis B;
    if (basis_build(&B, MOL_PASS)) { basis_free(&B); return -1; }
    for (int k = 0; k < 6 * B.sh_prim[nsh]; ++k) out[k] = (double)B.d[k];
    basis_free(&B);
    return 0;
}

int oracle_one_electron(MOL_ARGS, double *S, double *T, double *V)
{
    obasis B;
    if (basis_build(&B, MOL_PASS)) { basis_free(&B); return -1; }
    int N = B.nbf;
    #pragma omp parallel for schedule(dynamic)
    for (int sa = 0; sa < nsh; ++sa) {
        real s[36], t[36], v[36];
        for (int sb = 0; sb < nsh; ++sb) {
            one_electron_block(&B, sa, sb, s, t, v);
            int na = ncart(sh_l[sa]), nb = ncart(sh_l[sb]);
            for (int i = 0; i < na; ++i)
                for (int j = 0; j < nb; ++j) {
                    long idx = (long)(B.sh_bf[sa] + i) * N + B.sh_bf[sb] + j;
                    S[idx] = (double)s[i * nb + j]; T[idx] = (double)t[i * nb + j]; V[idx] = (double)v[i * nb + j];
                }
        }
    }
    basis_free(&B);
    return 0;
}

int oracle_eri_shell_quartet(MOL_ARGS, int a, int b, int c, int d, double *out)
{
    obasis B;
    if (basis_build(&B, MOL_PASS)) { basis_free(&B); return -1; }
    real blk[1296];
    eri_block(&B, a, b, c, d, blk);
    int n = ncart(sh_l[a]) * ncart(sh_l[b]) * ncart(sh_l[c]) * ncart(sh_l[d]);
    for (int k = 0; k < n; ++k) out[k] = (double)blk[k];
    basis_free(&B);
    return 0;
}

/* Blocks for a list of shell quartets; out_offsets[q] is where block q
 * starts in out (caller computes them). */
int oracle_eri_quartet_list(MOL_ARGS, long nq, const int *quartets, const long *out_offsets, double *out)
{
    obasis B;
    if (basis_build(&B, MOL_PASS)) { basis_free(&B); return -1; }
    #pragma omp parallel for schedule(dynamic)
    for (long q = 0; q < nq; ++q) {
        real blk[1296];
        const int *qq = quartets + 4 * q;
        eri_block(&B, qq[0], qq[1], qq[2], qq[3], blk);
        int n = ncart(sh_l[qq[0]]) * ncart(sh_l[qq[1]]) * ncart(sh_l[qq[2]]) * ncart(sh_l[qq[3]]);
        for (int k = 0; k < n; ++k) out[out_offsets[q] + k] = (double)blk[k];
    }
    basis_free(&B);
    return 0;
}

/* Full N^4 tensor; every shell quartet is evaluated on its own (no use of
 * permutational symmetry), so symmetry of the result is a genuine check. */
int oracle_eri_dense(MOL_ARGS, double *out)
{
    obasis B;
    if (basis_build(&B, MOL_PASS)) { basis_free(&B); return -1; }
    long N = B.nbf;
    #pragma omp parallel for schedule(dynamic)
    for (int ab = 0; ab < nsh * nsh; ++ab) {
        int sa = ab / nsh, sb = ab % nsh;
        real *blk = (real *)malloc(sizeof(real) * 1296);
        for (int sc = 0; sc < nsh; ++sc)
            for (int sd = 0; sd < nsh; ++sd) {
                eri_block(&B, sa, sb, sc, sd, blk);
                int na = ncart(sh_l[sa]), nb = ncart(sh_l[sb]), nc = ncart(sh_l[sc]), nd = ncart(sh_l[sd]);
                int k = 0;
                for (int i = 0; i < na; ++i)
                    for (int j = 0; j < nb; ++j)
                        for (int kk = 0; kk < nc; ++kk)
                            for (int ll = 0; ll < nd; ++ll, ++k) {
                                long i0 = B.sh_bf[sa] + i, j0 = B.sh_bf[sb] + j, k0 = B.sh_bf[sc] + kk, l0 = B.sh_bf[sd] + ll;
                                out[((i0 * N + j0) * N + k0) * N + l0] = (double)blk[k];
                            }
            }
        free(blk);
    }
    basis_free(&B);
    return 0;
}

/* Schwarz factors Q[a*nsh+b] = sqrt(max |(ab|ab)|) over the block. */
int oracle_schwarz(MOL_ARGS, double *Q)
{
    obasis B;
    if (basis_build(&B, MOL_PASS)) { basis_free(&B); return -1; }
    #pragma omp parallel for schedule(dynamic)
    for (int ab = 0; ab < nsh * nsh; ++ab) {
        int sa = ab / nsh, sb = ab % nsh;
        real *blk = (real *)malloc(sizeof(real) * 1296);
        eri_block(&B, sa, sb, sa, sb, blk);
        int na = ncart(sh_l[sa]), nb = ncart(sh_l[sb]);
        real m = 0.0;
        for (int i = 0; i < na * nb; ++i) {
            real v = fabs(blk[i * na * nb + i]);
            if (v > m) m = v;
        }
        Q[ab] = (double)sqrt(m);
        free(blk);
    }
    basis_free(&B);
    return 0;
}

/* J and K from unique shell quartets (a>=b, c>=d, ab>=cd) with the eight
 * permutation updates and the multiplicity factor
 * 1/((1+d_ab)(1+d_cd)(1+d_ab,cd)); quartets with Q_ab Q_cd < tau are
 * skipped (tau <= 0 keeps all).  D must be symmetric.  Returns the number of
 * quartets evaluated through *n_eval. */
int oracle_jk_unique(MOL_ARGS, const double *Dm, double tau, double *J, double *K, long long *n_eval)
{
    obasis B;
    if (basis_build(&B, MOL_PASS)) { basis_free(&B); return -1; }
    long N = B.nbf;
    int npair = nsh * (nsh + 1) / 2;
    int *pa = (int *)malloc(sizeof(int) * npair), *pb = (int *)malloc(sizeof(int) * npair);
    for (int a = 0, k = 0; a < nsh; ++a)
        for (int b = 0; b <= a; ++b, ++k) { pa[k] = a; pb[k] = b; }
    double *Q = (double *)malloc(sizeof(double) * nsh * nsh);
    if (tau > 0.0) oracle_schwarz(MOL_PASS, Q);
    memset(J, 0, sizeof(double) * N * N);
    memset(K, 0, sizeof(double) * N * N);
    long long count = 0;
    #pragma omp parallel reduction(+:count)
    {
        real *Jl = (real *)calloc(N * N, sizeof(real));
        real *Kl = (real *)calloc(N * N, sizeof(real));
        real *blk = (real *)malloc(sizeof(real) * 1296);
        #pragma omp for schedule(dynamic)
        for (int ab = npair - 1; ab >= 0; --ab) {
            int a = pa[ab], b = pb[ab];
            for (int cd = 0; cd <= ab; ++cd) {
                int c = pa[cd], d = pb[cd];
                if (tau > 0.0 && Q[a * nsh + b] * Q[c * nsh + d] < tau) continue;
                ++count;
                eri_block(&B, a, b, c, d, blk);
                real f = 1.0 / ((a == b ? 2.0 : 1.0) * (c == d ? 2.0 : 1.0) * (ab == cd ? 2.0 : 1.0));
                int na = ncart(sh_l[a]), nb = ncart(sh_l[b]), nc = ncart(sh_l[c]), nd = ncart(sh_l[d]);
                int k = 0;
                for (int ii = 0; ii < na; ++ii)
                for (int jj = 0; jj < nb; ++jj)
                for (int kk = 0; kk < nc; ++kk)
                for (int ll = 0; ll < nd; ++ll, ++k) {
                    long i = B.sh_bf[a] + ii, j = B.sh_bf[b] + jj, kx = B.sh_bf[c] + kk, l = B.sh_bf[d] + ll;
                    real v = f * blk[k];
                    /* (ij|kl) (ji|kl) (ij|lk) (ji|lk) (kl|ij) (lk|ij) (kl|ji) (lk|ji) */
                    Jl[i * N + j] += v * Dm[kx * N + l];  Kl[i * N + kx] += v * Dm[j * N + l];
                    Jl[j * N + i] += v * Dm[kx * N + l];  Kl[j * N + kx] += v * Dm[i * N + l];
                    Jl[i * N + j] += v * Dm[l * N + kx];  Kl[i * N + l] += v * Dm[j * N + kx];
                    Jl[j * N + i] += v * Dm[l * N + kx];  Kl[j * N + l] += v * Dm[i * N + kx];
                    Jl[kx * N + l] += v * Dm[i * N + j];  Kl[kx * N + i] += v * Dm[l * N + j];
                    Jl[l * N + kx] += v * Dm[i * N + j];  Kl[l * N + i] += v * Dm[kx * N + j];
                    Jl[kx * N + l] += v * Dm[j * N + i];  Kl[kx * N + j] += v * Dm[l * N + i];
                    Jl[l * N + kx] += v * Dm[j * N + i];  Kl[l * N + j] += v * Dm[kx * N + i];
                }
            }
        }
        #pragma omp critical
        {
            for (long x = 0; x < N * N; ++x) { J[x] += (double)Jl[x]; K[x] += (double)Kl[x]; }
        }
        free(Jl); free(Kl); free(blk);
    }
    *n_eval = count;
    free(pa); free(pb); free(Q);
    basis_free(&B);
    return 0;
}

/* Selected elements J[mu,nu] = sum (mu nu|ls) D[l,s] and
 * K[mu,nu] = sum (mu l|nu s) D[l,s], straight from the definitions. */
int oracle_jk_elements(MOL_ARGS, const double *Dm, int npts, const int *mu, const int *nu,
                       double *Jout, double *Kout)
{
    obasis B;
    if (basis_build(&B, MOL_PASS)) { basis_free(&B); return -1; }
    long N = B.nbf;
    int *bf_shell = (int *)malloc(sizeof(int) * N);
    for (int s = 0; s < nsh; ++s)
        for (int i = B.sh_bf[s]; i < B.sh_bf[s + 1]; ++i) bf_shell[i] = s;
    for (int e = 0; e < npts; ++e) {
        int m = mu[e], n = nu[e];
        int sm = bf_shell[m], sn = bf_shell[n];
        int im = m - B.sh_bf[sm], in_ = n - B.sh_bf[sn];
        real jsum = 0.0, ksum = 0.0;
        #pragma omp parallel for schedule(dynamic) reduction(+:jsum, ksum)
        for (int cd = 0; cd < nsh * nsh; ++cd) {
            int sc = cd / nsh, sd = cd % nsh;
            real *blk = (real *)malloc(sizeof(real) * 1296);
            int nm = ncart(sh_l[sm]), nnn = ncart(sh_l[sn]), nc = ncart(sh_l[sc]), nd = ncart(sh_l[sd]);
            /* J: (sm sn | sc sd) */
            eri_block(&B, sm, sn, sc, sd, blk);
            for (int kk = 0; kk < nc; ++kk)
                for (int ll = 0; ll < nd; ++ll)
                    jsum += blk[((im * nnn + in_) * nc + kk) * nd + ll]
                            * Dm[(B.sh_bf[sc] + kk) * N + B.sh_bf[sd] + ll];
            /* K: (sm sc | sn sd) */
            eri_block(&B, sm, sc, sn, sd, blk);
            for (int kk = 0; kk < nc; ++kk)
                for (int ll = 0; ll < nd; ++ll)
                    ksum += blk[((im * nc + kk) * nnn + in_) * nd + ll]
                            * Dm[(B.sh_bf[sc] + kk) * N + B.sh_bf[sd] + ll];
            free(blk);
        }
        Jout[e] = (double)jsum; Kout[e] = (double)ksum;
    }
    free(bf_shell);
    basis_free(&B);
    return 0;
}
