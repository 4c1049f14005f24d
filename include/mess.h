/*
 * mess.h — C ABI of the MI355X (gfx950) Gaussian-basis Hartree-Fock hot path.
 *
 * The library computes what section 3 of the MESS paper ("Electronic
 * Structure Theory in a Nutshell") states as the problem: given atoms
 * (atomic numbers and positions) and a basis of contracted Gaussian atomic
 * orbitals on them (eq. 1), build the overlap matrix (eq. 3) and the other
 * closed-form Gaussian integrals, the Coulomb/exchange matrices J and K from
 * a density matrix, and iterate the Roothaan equation (eq. 2) to
 * self-consistency, returning energies (electronic + nuclear, as in the
 * paper's examples of section 5).
 *
 * Conventions (all entry points):
 *  - Units: bohr and hartree.
 *  - Basis: contracted Cartesian shells with l in {0,1,2}.  Components of a
 *    shell are ordered x-major lexicographically (p: x,y,z; d: xx,xy,xz,yy,
 *    yz,zz) and every Cartesian function is normalised to unit
 *    self-overlap.  Contraction coefficients multiply normalised
 *    primitives; the contracted function is then renormalised.
 *  - Basis functions are numbered shell by shell in the order given.
 *  - Matrices are N x N, row-major, contiguous, FP64, in DEVICE memory
 *    (hipMalloc'd or torch CUDA tensors).  Atom and shell arrays are HOST
 *    memory and are copied at create time.
 *  - D is the total closed-shell density, D = 2 C_occ C_occ^T (symmetric).
 *  - J_ij = sum_kl (ij|kl) D_kl,   K_ij = sum_kl (ik|jl) D_kl.
 *  - Every call returns a status code.  On error nothing is written to
 *    outputs that were not already written, handles stay valid and usable,
 *    and mess_last_error() returns a message (thread-local).
 *  - Work is enqueued on `stream` (a hipStream_t, NULL = null stream).
 *    Calls that return host scalars (mess_basis_info, mess_scf_step)
 *    synchronise that stream; the others do not.
 *  - A handle must not be used from two threads at once.
 */
#ifndef MESS_H
#define MESS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mess_basis mess_basis;
typedef struct mess_scf mess_scf;
typedef struct mess_batch_scf mess_batch_scf;
typedef struct mess_mlp mess_mlp;
typedef void *mess_stream;

enum {
    MESS_OK = 0,
    MESS_E_ARG = 1,          /* NULL pointer, out-of-range index, non-positive or non-finite value */
    MESS_E_UNSUPPORTED = 2,  /* l > 2, odd electron count, unknown mode */
    MESS_E_NOMEM = 3,        /* device allocation failed */
    MESS_E_DEVICE = 4,       /* HIP runtime error */
    MESS_E_NUMERIC = 5,      /* ill-conditioned overlap, NaN in a result */
    MESS_E_SIZE = 6          /* output buffer too small */
};

enum { MESS_FP64 = 0, MESS_FP32 = 1 };                       /* arithmetic of the ERI path */
enum { MESS_ERI_DENSE = 0, MESS_ERI_BLOCKS = 1 };            /* mess_eri output layout */
enum { MESS_JK_DIRECT = 0, MESS_JK_STORED = 1,               /* mess_jk source of integrals */
       MESS_JK_DETERMINISTIC = 2 };                          /* stored blocks, exact accumulation */
enum { MESS_XC_HF = 0, MESS_XC_LDA_X = 1, MESS_XC_PBE = 2 };  /* exchange(-correlation) in the Fock matrix */

typedef struct mess_scf_opts {
    double schwarz_tol;  /* skip quartet iff Q_ab Q_cd < tol; <= 0 keeps every quartet */
    double conv_tol;     /* converged when |E_k - E_{k-1}| < conv_tol */
    int32_t max_iter;    /* informational for callers driving mess_scf_step */
    int32_t diis_size;   /* Pulay DIIS history length; 0 = plain Roothaan iteration */
    int32_t prec;        /* MESS_FP64, or MESS_FP32 (mixed precision): until |dE| first
                            drops below 0.1 Ha every Fock build is a complete FP32 build;
                            the first build after that is a complete FP64 build, the next ones
                            build dD = D_k - D_{k-1} in FP32 and add it to the FP64 J/K,
                            with a complete FP64 rebuild after every 8 of them.  With
                            MESS_JK_DIRECT and schwarz_tol > 0 the dD builds also skip
                            quartets with Q_ab Q_cd max|dD| < schwarz_tol (threshold
                            rounded down to a power of ten).  Convergence is declared only
                            on two successive FP64-anchored energies.  Energies,
                            eigen-problem and density in FP64; classes whose FP64 kernel is
                            faster run in FP64 (MESS_FORM_FP64) */
    int32_t jk_mode;     /* MESS_JK_DIRECT or MESS_JK_STORED */
    int32_t xc;          /* MESS_XC_HF (F = H + J - K/2), MESS_XC_LDA_X (F = H + J + V_x,
                            E = Tr[D H] + 1/2 Tr[D J] + E_x + E_nuc; see mess_lda_x) or
                            MESS_XC_PBE (the same with V_xc, E_xc of mess_pbe_xc); the
                            last two FP64 only */
    int32_t deterministic; /* nonzero: every Fock build runs as mess_jk(MESS_JK_DETERMINISTIC)
                              (overrides jk_mode), so a rerun reproduces every energy and
                              density bit for bit */
    int32_t no_guard;    /* nonzero: no divergence guard.  The guard (default): an energy
                            rise above 1e-6 Ha counts against the current stage and the
                            second rise in a stage moves to the next; a non-finite energy
                            goes straight to the last.  Each change drops the DIIS history.
                            Stages: 0 DIIS; 1 DIIS afresh; 2 DIIS with the next density
                            mixed half and half with the current one; 3 restart from the
                            core-Hamiltonian guess, damped as in 2 (the first energy after
                            the restart is compared with nothing).  A non-finite energy in
                            stage 3, or with the guard off, is MESS_E_NUMERIC */
} mess_scf_opts;

/* Build a basis on a molecule (section 3, eq. 1: each atomic orbital sits
 * on one atom with centre R and atomic number Z).
 *   n_atoms, Z[n_atoms], xyz_bohr[3*n_atoms]          host arrays
 *   n_shells, shell_atom/shell_l/shell_nprim[n_shells] host arrays
 *   exps[sum nprim] > 0, coefs[sum nprim] (raw contraction coefficients)
 *   charge: molecular charge (electrons = sum Z - charge)
 * Normalises the basis, builds primitive-pair tables, Schwarz factors of
 * every shell pair and nuclear repulsion, on the device.  Primitive pairs
 * whose Coulomb bound U_uv (a Gaussian majorant of the primitive product;
 * |(uv|wx)| <= U_uv U_wx for every component) times the largest bound is
 * below 1e-14 / (2 npp_max^2) are left out (npp_max: the most primitive
 * pairs of one shell pair), so no contracted integral moves by more than
 * 1e-14; every shell pair keeps at least its largest term.
 * Errors: MESS_E_ARG (NULL, index out of range, exponent <= 0 or not
 * finite, nprim < 1 or > 16), MESS_E_UNSUPPORTED (l > 2), MESS_E_NOMEM. */
int mess_basis_create(int32_t n_atoms, const int32_t *Z, const double *xyz_bohr,
                      int32_t n_shells, const int32_t *shell_atom, const int32_t *shell_l,
                      const int32_t *shell_nprim, const double *exps, const double *coefs,
                      int32_t charge, mess_basis **out);

/* A batch of independent molecules in one basis handle, so that the
 * shell quartets of every molecule share one launch per angular class
 * (the paper's batching of many small systems, section 5).  Molecules are
 * given back to back: molecule m has mol_atoms[m] atoms and
 * mol_shells[m] shells; Z, xyz_bohr, shell_atom, shell_l, shell_nprim,
 * exps and coefs are the concatenation of the per-molecule arrays of
 * mess_basis_create, with shell_atom indices local to each molecule.
 * charges[n_mol] may be NULL (all neutral).  Host arrays, copied.
 * Functions are numbered molecule by molecule.  Every matrix of a batch
 * handle is PACKED BLOCK-DIAGONAL: molecule m's nbf_m x nbf_m row-major
 * block at element offset moff[m] (mess_batch_info), total moff[n_mol]
 * doubles; mess_one_electron and mess_jk read and write this layout.
 * Quartets never couple two molecules.  mess_eri and mess_scf_create
 * reject a batch of more than one molecule (MESS_E_UNSUPPORTED / _ARG).
 * Errors: as mess_basis_create, and MESS_E_ARG if the per-molecule counts
 * do not cover the arrays. */
int mess_batch_create(int32_t n_mol, const int32_t *mol_atoms, const int32_t *mol_shells,
                      const int32_t *charges, const int32_t *Z, const double *xyz_bohr,
                      const int32_t *shell_atom, const int32_t *shell_l, const int32_t *shell_nprim,
                      const double *exps, const double *coefs, mess_basis **out);

/* Per-molecule layout of a basis handle (a single molecule is a batch of
 * one): n_mol; nbf[n_mol]; moff[n_mol + 1] packed offsets; n_occ[n_mol];
 * e_nuc[n_mol].  Host outputs, any may be NULL (arrays sized by the
 * caller from a first call with only n_mol). */
int mess_batch_info(const mess_basis *basis, int32_t *n_mol, int32_t *nbf, int64_t *moff,
                    int32_t *n_occ, double *e_nuc);

/* Frees every device allocation of the handle.  NULL is a no-op. */
void mess_basis_destroy(mess_basis *basis);

/* Number of basis functions, occupied orbitals (electrons/2, rounded
 * down) and nuclear repulsion sum_{A<B} Z_A Z_B / R_AB.  Any output may be
 * NULL.  Synchronous. */
int mess_basis_info(const mess_basis *basis, int32_t *nbf, int32_t *n_occ, double *e_nuc);

/* One-electron matrices (section 3, eq. 3 for S; kinetic T and nuclear
 * attraction V for the core Hamiltonian H = T + V).  Each output is a
 * device N x N buffer or NULL to skip. */
int mess_one_electron(const mess_basis *basis, double *S, double *T, double *V, mess_stream stream);

/* J and K of ndens densities from a dense ERI tensor (section 3: Coulomb
 * and exchange matrices are contractions of the repulsion integrals with
 * the density):
 *   J[d][i][j] = sum_kl (ij|kl) D[d][k][l],  K[d][i][j] = sum_kl (ik|jl) D[d][k][l],
 * as products over the composite indices (ij), (kl) of the n^2 x n^2 view
 * of the tensor.  eri: device n^4 elements, row-major ((i n + j) n + k) n + l
 * (mess_eri MESS_ERI_DENSE, full tensor); D, J, K: device [ndens][n][n]
 * (J or K may be NULL).  prec MESS_FP64 (double arrays) or MESS_FP32 (float
 * arrays, FP32 accumulation).  form MESS_DENSE_MFMA (matrix cores, 16x16x4
 * products) or MESS_DENSE_VALU (vector FMAs, the same tiling).
 * Asynchronous.  Errors: MESS_E_ARG (NULL eri or D, n < 1, ndens < 1,
 * unknown prec or form). */
enum { MESS_DENSE_VALU = 0, MESS_DENSE_MFMA = 1 };
int mess_jk_dense(const void *eri, int32_t n, int32_t ndens, const void *D, void *J, void *K, int32_t prec,
                  int32_t form, mess_stream stream);

/* Boys function F_j(T) = int_0^1 u^(2j) exp(-T u^2) du, j = 0..m (section 3:
 * every closed-form repulsion integral is a sum over it), by the device
 * routines of the integral kernels, using the basis handle's tables:
 *   form 0  F_0..F_m together (Taylor sum of F_m about T_k = k/16, downward
 *           recurrence; (2j-1)!!/(2T)^j sqrt(pi/T)/2 for T >= 60), the
 *           recursion kernels' form;
 *   form 1  each F_j by its own Taylor sum, the table-driven kernel's form.
 * prec MESS_FP64, or MESS_FP32 for the mixed-precision kernels' FP32 forms
 * (T rounded to FP32, results widened).  T: device, n doubles, T >= 0 (a
 * negative or NaN T gives NaN); F: device, n * (m + 1) doubles,
 * F[i * (m + 1) + j] = F_j(T[i]).  0 <= m <= 8.  Asynchronous on stream.
 * Errors: MESS_E_ARG (NULL pointers with n > 0, m, form or prec out of
 * range). */
int mess_boys(const mess_basis *basis, int32_t prec, int32_t form, int32_t m, const double *T, int64_t n,
              double *F, mess_stream stream);

/* Electron-repulsion integrals (mu nu|lambda sigma) over the basis: the
 * four-centre Coulomb integrals of pairs of basis functions (section 3,
 * eq. 1 basis functions; the closed-form Gaussian integrals the section
 * lists with the overlap of eq. 3).
 *   layout MESS_ERI_DENSE: out is a device N^4 FP64 tensor (i slowest);
 *     every element is written (screened quartets are zero).
 *     out_bytes must be >= 8 N^4.  Single molecules only.  prec MESS_FP32
 *     computes in FP32 and stores widened to FP64.
 *   layout MESS_ERI_BLOCKS: the unique shell quartets (ab|cd), pair (ab)
 *     >= pair (cd), that pass the Schwarz test, class by class in the order
 *     cls = cb (cb + 1) / 2 + ck (pair classes ss ps pp ds dp dd = 0..5);
 *     within class cls, element k = ((a NB + b) NC + c) ND + d of its
 *     quartet t (a, b, c, d Cartesian components of the four shells, NA..ND
 *     their counts) at out[off_cls + k nq_cls + t], off_cls the sum of
 *     NA NB NC ND nq over the earlier classes.  Elements are FP64, or FP32
 *     with prec MESS_FP32.  mess_eri_quartets gives nq_cls and the shells
 *     of every quartet.  Works for batches too (quartets of one molecule).
 *   schwarz_tol: skip quartet iff Q_ab Q_cd < tol (<= 0 keeps all).
 * Errors: MESS_E_SIZE, MESS_E_UNSUPPORTED (layout), MESS_E_ARG. */
int mess_eri(const mess_basis *basis, int32_t layout, int32_t prec, double schwarz_tol,
             void *out, size_t out_bytes, mess_stream stream);

/* Unique shell quartets of the MESS_ERI_BLOCKS layout (host outputs, either
 * may be NULL): counts[21] quartets per class; shells[sum counts][4] the
 * shell indices (a, b, c, d) of every quartet in output order (shells
 * numbered as given at create, across a batch). */
int mess_eri_quartets(const mess_basis *basis, double schwarz_tol, int64_t *counts, int32_t *shells);

/* Coulomb and exchange matrices from a symmetric density D (device N x N):
 *   J_ij = sum_kl (ij|kl) D_kl,  K_ij = sum_kl (ik|jl) D_kl,
 * the two-electron parts of the Fock operator of the Roothaan equation
 * (section 3, eq. 2; K is the exact (Hartree-Fock) exchange the paper's
 * examples select as the exchange functional, section 5.1).
 * J or K may be NULL to skip.  mode MESS_JK_DIRECT recomputes integrals
 * over unique shell quartets (8-fold permutational symmetry) with Schwarz
 * screening and digests them in registers; MESS_JK_STORED computes the
 * unique blocks once per (basis, prec, tol) and streams them from device
 * memory on later calls; MESS_JK_DETERMINISTIC digests the same stored
 * blocks with exact 128-bit fixed-point accumulation (resolution 2^-80),
 * so repeated calls return bitwise equal J and K (synchronous;
 * MESS_E_NUMERIC if a contribution exceeds 2^46).  prec selects FP64 or
 * FP32 integral arithmetic (J, K are always returned in FP64). */
int mess_jk(const mess_basis *basis, const double *D, double *J, double *K,
            int32_t mode, int32_t prec, double schwarz_tol, mess_stream stream);

/* mess_jk in MESS_JK_DIRECT mode for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same kernels and results as mess_jk, but the J/K
 * half matrices live in a fixed device array of the library (2 x 2^19
 * doubles, 8 MB per device, held until the process ends) instead of the
 * basis handle's buffer, and the call allocates and frees nothing.
 *   D, J, K as for mess_jk (J or K may be NULL); prec MESS_FP64 or
 *   MESS_FP32; schwarz_tol as for mess_jk.
 * The work lists for (basis, schwarz_tol) must already exist: call mess_jk
 * once with the same basis and tolerance first (MESS_E_ARG otherwise).
 * MESS_E_SIZE if the basis has more than 2^19 matrix elements (N > 724,
 * or a batch whose packed matrices exceed that).  MESS_E_ARG while class
 * profiling is on.  All calls on one device share the array: calls that
 * overlap in time on one device (two streams, two threads) race; calls
 * ordered on one stream do not. */
int mess_jk_noalloc(const mess_basis *basis, const double *D, double *J, double *K, int32_t prec,
                    double schwarz_tol, mess_stream stream);

/* LDA exchange (the local density approximation the paper names for its
 * batched DFT example, section 5), as Dirac-Slater exchange on an
 * atom-centred grid:
 *   rho_g = sum_{mu nu} phi_mu(r_g) D_{mu nu} phi_nu(r_g),
 *   E_x = -(3/4)(3/pi)^(1/3) sum_g w_g rho_g^(4/3),
 *   V_x[mu][nu] = -(3/pi)^(1/3) sum_g w_g rho_g^(1/3) phi_mu(r_g) phi_nu(r_g)
 * (points with rho_g <= 0 contribute nothing).  Grid per atom: 75 radial
 * nodes (second-kind Gauss-Chebyshev, x_i = cos(i pi/76), r = (1+x)/(1-x)
 * bohr) times 17 Gauss-Legendre nodes in cos(theta) times 34 azimuths,
 * Becke fuzzy-cell weights (three iterations of f(x) = (3x - x^3)/2);
 * 43,350 points per atom.  The grid and the basis values on it are built on
 * the first call (synchronous, 8 N bytes per point) and kept in the basis.
 *   D: device N x N symmetric density.  Vx: device N x N or NULL.
 *   Ex: host scalar or NULL (non-NULL synchronises the stream).
 *   rho: device array of mess_grid's point count, or NULL.
 * Errors: MESS_E_UNSUPPORTED for a batch of more than one molecule,
 * MESS_E_NOMEM. */
int mess_lda_x(const mess_basis *basis, const double *D, double *Vx, double *Ex, double *rho,
               mess_stream stream);

/* PBE exchange-correlation (the generalised-gradient functional the paper
 * selects through its Hamiltonian's exchange-correlation option, section
 * 5; Perdew, Burke and Ernzerhof 1996), closed shell, on the grid of
 * mess_lda_x:
 *   sigma = |grad rho|^2, grad rho_g = 2 sum_{mu nu} D_{mu nu} phi_mu grad phi_nu,
 *   f = rho eps_x^unif F_x(s) + rho (eps_c^PW92(r_s) + H(r_s, t)),
 *   E_xc = sum_g w_g f_g,
 *   V_xc[mu][nu] = sum_g w_g [f_rho phi_mu phi_nu
 *                   + 2 f_sigma grad rho . grad(phi_mu phi_nu)]
 * with kappa = 0.804, beta = 0.06672455060314922, mu = beta pi^2/3,
 * gamma = (1 - ln 2)/pi^2 and the Perdew-Wang (1992) paramagnetic
 * correlation (A = 0.031091, a1 = 0.21370, b = 7.5957, 3.5876, 1.6382,
 * 0.49294); points with rho < 1e-10 contribute nothing.  The basis
 * gradients on the grid are built on the first call (24 N bytes per point
 * beyond mess_lda_x's) and kept in the basis.
 *   D: device N x N symmetric density.  Vxc: device N x N or NULL.
 *   Exc: host scalar or NULL (non-NULL synchronises the stream).
 *   rho: device [npts] or NULL; grad_rho: device [3][npts] or NULL.
 * Errors: MESS_E_UNSUPPORTED for a batch of more than one molecule,
 * MESS_E_NOMEM. */
int mess_pbe_xc(const mess_basis *basis, const double *D, double *Vxc, double *Exc, double *rho,
                double *grad_rho, mess_stream stream);

/* The LDA grid: *npts points (host, may be NULL); xyzw (device, may be
 * NULL) receives [npts][4] = x, y, z (bohr) and weight, ordered by atom,
 * radial node (largest radius first), theta node (ascending cos theta),
 * azimuth 2 pi k / 34. */
int mess_grid(const mess_basis *basis, double *xyzw, int64_t *npts, mess_stream stream);

/* SCF state for the Roothaan equation (section 3, eq. 2) solved by
 * fixed-point iteration.  D0: device N x N initial density, or NULL for
 * the core-Hamiltonian guess.  Errors: MESS_E_UNSUPPORTED (odd electron
 * count), MESS_E_NUMERIC (overlap too ill-conditioned: lambda_min(S)
 * below about 1e-7). */
int mess_scf_create(const mess_basis *basis, const mess_scf_opts *opts, const double *D0,
                    mess_scf **out);

/* One SCF iteration at the current density D_k:
 *   J, K <- D_k;  F_k = H + J - K/2;  E_k = 1/2 Tr[D_k (H + F_k)] + E_nuc;
 *   converged = (k > 0 and |E_k - E_{k-1}| < conv_tol);
 *   unless converged: DIIS-extrapolated F (if diis_size > 0, once two
 *   Fock matrices are stored, error X^T (F D S - S D F) X), then
 *   D_{k+1} = projector onto the n_occ lowest eigenvectors of F in the
 *   metric S (times 2) becomes the current density.
 * Outputs (host, any may be NULL): energy E_k, delta_e = E_k - E_{k-1}
 * (0 at k = 0), resid = max |X^T (F D S - S D F) X|, converged flag.
 * Synchronises the stream.  Non-convergence is not an error. */
/* Nuclear gradient dE/dR of the closed-shell Hartree-Fock energy (the
 * atomic forces the paper obtains by differentiating its energy, sections
 * 1 and 4), analytic:
 *   dE/dR_X = sum D dH/dR_X + 1/2 sum P d(mu nu|la si)/dR_X
 *             - sum W dS/dR_X + dE_nuc/dR_X,
 * W = D F D / 2, P = D_{mu nu} D_{la si} - (D_{mu la} D_{nu si} + D_{mu si} D_{nu la}) / 4,
 * with the integral derivatives from Hermite expansions one order above
 * the differentiated function.  Valid at a converged density (D and F of
 * the same SCF iteration; the energy must be stationary in D).
 *   D, F: device N x N.  schwarz_tol: shell quartets with Q_ab Q_cd below
 *   it are left out (0 keeps all).  grad: host [n_atoms][3], Hartree/bohr.
 * Synchronous.  Errors: MESS_E_ARG (NULL), MESS_E_UNSUPPORTED (a batch of
 * more than one molecule), MESS_E_NOMEM. */
int mess_hf_gradient(const mess_basis *basis, const double *D, const double *F, double schwarz_tol,
                     double *grad, mess_stream stream);

/* mess_hf_gradient at the handle's current density and Fock matrix, to be
 * called after the step that reported convergence (Hartree-Fock only:
 * MESS_E_UNSUPPORTED otherwise). */
int mess_scf_gradient(const mess_scf *scf, double *grad, mess_stream stream);

/* Divergence-guard stage of the run (0..3, see mess_scf_opts.no_guard) and
 * the energy rises counted in it.  Host outputs, either may be NULL. */
int mess_scf_guard(const mess_scf *scf, int32_t *stage, int32_t *rises);

int mess_scf_step(mess_scf *scf, double *energy, double *delta_e, double *resid,
                  int32_t *converged, mess_stream stream);

/* Direct minimisation of the energy (section 3: minimise E(C) subject to
 * the orthonormality constraint C^T S C = 1 of eq. 5, the constraint built
 * in by QR orthonormalisation of an unconstrained trial matrix; section 5.1:
 * first-order optimisation with Adam from Z = 1).  One step on an SCF
 * handle: Z = Q R, C = X Q with X = S^{-1/2}, D = 2 C_occ C_occ^T (C_occ the
 * first n_occ columns), E = 1/2 Tr[D (H + F)] + E_nuc with F from a Fock
 * build in the handle's J/K mode and precision; the gradient
 * dE/dZ = Q tril(B^T - B, -1) R^{-T}, B = (X^T 4 F C_occ)^T Q (zero beyond
 * column n_occ); then one Adam update of Z (lr, beta1 0.9, beta2 0.999,
 * eps 1e-8, bias-corrected).  The first call starts from Z = 1.  Outputs
 * (host, may be NULL): E of the Z before the update, max |dE/dZ|.  The
 * handle's density and Fock matrix become those of that Z.  Synchronous.
 * Errors: MESS_E_ARG (lr not positive), MESS_E_UNSUPPORTED (LDA exchange,
 * or an overlap that needed the canonical orthogonaliser), MESS_E_NUMERIC
 * (Z became singular, or a non-finite result). */
int mess_dmin_step(mess_scf *scf, double lr, double *energy, double *grad_max, mess_stream stream);
/* The energy E(Z) (host, may be NULL) and its gradient dE/dZ (device N x N,
 * may be NULL) of mess_dmin_step for a given trial matrix Z (device N x N),
 * with no optimiser update.  Synchronous.  Errors as mess_dmin_step. */
int mess_dmin_eval(mess_scf *scf, const double *Z, double *energy, double *G, mess_stream stream);
/* Copy the current trial matrix Z (device N x N) of a handle that has taken
 * direct-minimisation steps. */
int mess_dmin_trial(const mess_scf *scf, double *Z, mess_stream stream);

/* Copy the current density (device N x N) into D. */
int mess_scf_density(const mess_scf *scf, double *D, mess_stream stream);

/* Copy the Fock matrix of the last step (device N x N) into F. */
int mess_scf_fock(const mess_scf *scf, double *F, mess_stream stream);

/* NULL is a no-op. */
void mess_scf_destroy(mess_scf *scf);

/* Batched SCF over every molecule of a batch handle: the step of
 * mess_scf_step applied to each molecule, with all molecules' ERI classes,
 * Fock builds, DIIS and density purifications sharing launches.
 * opts->prec MESS_FP64, or MESS_FP32 (mixed precision decided by the step
 * count alone, so steps stay free of host decisions): the first 2 Fock
 * builds are complete FP32 builds, the third a complete FP64 build, later
 * ones FP32 builds of the density change added to it with a complete FP64
 * rebuild after every 8; a molecule freezes only on two successive
 * FP64-anchored energies.  X is the Loewdin S^{-1/2} of each
 * molecule (MESS_E_NUMERIC if an overlap block may be near-singular).
 * D0: device packed initial density, or NULL for the core-Hamiltonian
 * guess.  use_graph != 0 captures the first step into a HIP graph and
 * replays it on later steps (the caller's stream must not be capturing;
 * class profiling must be off).  Builds the work lists (and, for
 * MESS_JK_STORED, the stored integrals) before returning, so that a step
 * allocates nothing.  Synchronous. */
int mess_batch_scf_create(const mess_basis *basis, const mess_scf_opts *opts, const double *D0,
                          int32_t use_graph, mess_batch_scf **out);

/* Enqueue one SCF iteration for every molecule on the stream; does not
 * synchronise.  A molecule with k > 0 and |E_k - E_{k-1}| < conv_tol is
 * frozen: its energy and density stay those of that step.  The divergence
 * guard of mess_scf_opts.no_guard runs per molecule (a molecule restarting
 * after a non-finite energy keeps its last finite energy in the status;
 * in stage 3 a non-finite energy freezes it, and the status reports it). */
int mess_batch_scf_step(mess_batch_scf *scf, mess_stream stream);

/* Divergence-guard stage (0..3) of every molecule: stage[n_mol], host.
 * Synchronous. */
int mess_batch_scf_guard(const mess_batch_scf *scf, int32_t *stage);

/* Synchronise and read per-molecule results of the last step (host arrays
 * of n_mol, any may be NULL): energy, delta_e, resid, converged flag, and
 * the number converged.  MESS_E_NUMERIC if an energy is not finite or a
 * density purification did not finish. */
int mess_batch_scf_status(const mess_batch_scf *scf, double *energy, double *delta_e, double *resid,
                          int32_t *converged, int32_t *n_converged, mess_stream stream);

/* Copy the current packed density into D (device). */
int mess_batch_scf_density(const mess_batch_scf *scf, double *D, mess_stream stream);

/* NULL is a no-op. */
void mess_batch_scf_destroy(mess_batch_scf *scf);

/* ---- Learned initial guess ----
 * The paper writes its energies as differentiable programs so that learned
 * components can be fitted to data (sections 1 and 5); here a perceptron
 * predicts the initial density from atom-pair features.
 *
 * Pair rows: for each molecule of a basis (single or batch), atom pairs
 * A <= B in A-major order.  Features, float [rows][64] (42 used): one-hot
 * element of A and of B over (H, C, N, O); 16 Gaussians
 * exp(-((R_AB - 2k/3)/(2/3))^2), k = 0..15; unit vector A->B and its six
 * products (xx, xy, xz, yy, yz, zz), zero for A = B; per-element counts of
 * the other atoms around A and around B weighted by (cos(pi R/6) + 1)/2
 * below R = 6 bohr; a self-pair flag.  Outputs, float [rows][128]: element
 * 11 i + j is the density between function i of A and function j of B
 * (atoms carry 1..11 functions, contiguous; H, C, N, O only, else
 * MESS_E_UNSUPPORTED).
 *
 * Perceptron 64 -> 256 -> 256 -> 128, SiLU on both hidden layers.  FP32
 * parameters, MESS_MLP_NPARAM floats in the order W1 [256][64], b1[256],
 * W2 [256][256], b2[256], W3 [128][256], b3[128] (y = W x + b).  Every layer
 * product runs on the BF16 matrix cores: operands (inputs, weights,
 * activations, back-propagated gradients) rounded to BF16 (nearest, ties
 * to even), FP32 accumulation; biases, pre-activations and gradients FP32.
 * Training loss: mean of M (Y - T)^2 over the elements with mask M = 1;
 * Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on FP32 masters.
 * All row arrays are device pointers; at most 2^21 rows per call. */
enum { MESS_MLP_IN = 64, MESS_MLP_HIDDEN = 256, MESS_MLP_OUT = 128, MESS_MLP_NPARAM = 115328 };

/* params: host, MESS_MLP_NPARAM floats (copied).  Adam moments start at 0. */
int mess_mlp_create(const float *params, mess_mlp **out);
void mess_mlp_destroy(mess_mlp *mlp);
/* Copy the FP32 parameters to host params[MESS_MLP_NPARAM] (synchronous). */
int mess_mlp_params(const mess_mlp *mlp, float *params);
/* Y[n][128] = perceptron(X[n][64]). */
int mess_mlp_forward(mess_mlp *mlp, int64_t n, const float *X, float *Y, mess_stream stream);
/* Gradient of the masked loss into grad[MESS_MLP_NPARAM] (device, may be
 * NULL) and the loss into *loss (host, may be NULL; synchronises). */
int mess_mlp_grad(mess_mlp *mlp, int64_t n, const float *X, const float *T, const float *M, float *grad,
                  double *loss, mess_stream stream);
/* Gradient, then one Adam step with learning rate lr > 0. */
int mess_mlp_train_step(mess_mlp *mlp, int64_t n, const float *X, const float *T, const float *M, float lr,
                        double *loss, mess_stream stream);

/* Number of pair rows of a basis (host output). */
int mess_guess_rows(const mess_basis *basis, int64_t *n_rows);
/* Features of every pair row into X (device [rows][64]). */
int mess_guess_features(const mess_basis *basis, float *X, mess_stream stream);
/* Training targets from a density (device, packed): T = the pair blocks of
 * D, M = 1 inside each block; either may be NULL. */
int mess_guess_targets(const mess_basis *basis, const double *D, float *T, float *M, mess_stream stream);
/* Density (device, packed) from outputs Y: D[A_i][B_j] = D[B_j][A_i] =
 * Y[11 i + j]; diagonal blocks take the mean of Y[11 i + j] and Y[11 j + i]. */
int mess_guess_assemble(const mess_basis *basis, const float *Y, double *D, mess_stream stream);
/* In place: D <- 2 S^-1/2 V V^T S^-1/2 per molecule, V the n_occ
 * eigenvectors of S^1/2 D S^1/2 of largest eigenvalue (idempotent in the
 * metric S, trace N_e), computed with the Loewdin S^-1/2 and the batched
 * purification.  Synchronous.  MESS_E_NUMERIC if purification fails. */
int mess_guess_project(const mess_basis *basis, double *D, mess_stream stream);
/* Per molecule, keep D0's block if its first commutator residual
 * max |X^T (F D S - S D F) X| (Hartree-Fock F, opts as for
 * mess_batch_scf_create) is below the core-Hamiltonian guess's, else
 * replace it by the core guess; used[n_mol] (host, may be NULL) receives
 * 1 where D0 was kept.  Synchronous. */
int mess_guess_judge(const mess_basis *basis, const mess_scf_opts *opts, double *D0, int32_t *used,
                     mess_stream stream);

/* ---- Instrumentation (not part of the method; used by benchmarks). ----
 * Class index cls = cb (cb + 1) / 2 + ck for bra pair class cb >= ket pair
 * class ck, pair classes ss, ps, pp, ds, dp, dd = 0..5.
 *
 * mess_work_stats: for the unique, Schwarz-screened shell-quartet list of
 * one class: number of shell quartets, of primitive quartets, and the
 * algorithmic FP64 operation count of one direct J/K pass over it (an FMA
 * counts 2; Boys function, vertical and horizontal recursion, contraction
 * and J/K digestion).  Host outputs, any may be NULL.
 *
 * mess_prof_enable(1) starts recording a pair of HIP events on the launch
 * stream around every class launch of mess_jk / mess_scf_step (0 stops;
 * both discard earlier records).  Direct launches in FP32 arithmetic are
 * recorded under cls + 64, stored-block streams under cls + 32.  mess_prof_read sums, for one class (or
 * all with cls = -1), launches, elapsed milliseconds between the events,
 * algorithmic operations, shell and primitive quartets.  Synchronises on
 * the recorded events. */
int mess_work_stats(const mess_basis *basis, double schwarz_tol, int32_t cls, int64_t *quartets,
                    int64_t *prim_quartets, double *alg_flops_jk);
/* Primitive pairs of the basis kept by the screening of mess_basis_create,
 * and the count before it.  Host outputs, either may be NULL. */
int mess_prim_pairs(const mess_basis *basis, int64_t *kept, int64_t *full);
int mess_prof_enable(int32_t on);
int mess_prof_read(int32_t cls, int64_t *launches, double *ms, double *alg_flops, int64_t *quartets,
                   int64_t *prim_quartets);

/* ---- Kernel forms and the autotuner ----
 * Each angular class can run in several mappings onto the GPU:
 *   MESS_FORM_LANE   one lane per shell quartet (recursion in registers);
 *   MESS_FORM_ROWS   one block per segment of a bra's quartets, exchange rows
 *                    of the bra functions accumulated in LDS (low classes);
 *   MESS_FORM_PLANE  one wave per shell quartet, one lane per primitive
 *                    quartet, intermediates summed across the wave;
 *   MESS_FORM_COOP   one block per shell quartet, the recursion table-driven
 *                    in LDS (high classes);
 *   MESS_FORM_WAVE   one block per shell quartet, one wave per primitive
 *                    quartet, lanes over the recursion's intermediates, the
 *                    contracted outputs kept in registers ((dd|ds), (dd|dp),
 *                    (dd|dd));
 *   MESS_FORM_FP64   FP32 table only: direct J/K builds asked for in FP32
 *                    evaluate the class with its FP64 kernel (more accurate,
 *                    and faster for the low classes on this hardware).
 * The choice is process-wide, kept per precision of the integral arithmetic
 * (MESS_FP64, MESS_FP32), and applies to every later launch in that
 * precision (mess_eri, mess_jk, SCF and batch steps).
 *
 * mess_kernel_form: set the form of class cls (index as for
 * mess_work_stats) in precision prec when form >= 0 (MESS_FORM_AUTO
 * restores the built-in default), and return the active form in *active
 * (may be NULL).  MESS_E_UNSUPPORTED if the form is not built for the
 * class, MESS_E_ARG for an unknown precision or class.
 *
 * mess_autotune: for every class with quartets in the basis's work list at
 * schwarz_tol, time each available form in precision prec on a direct J/K
 * pass with density D
 * (device N x N, or packed for a batch) as the best of reps runs after one
 * warm-up (HIP events on the stream), and keep the fastest.  forms[21]
 * (host, may be NULL) receives the chosen forms; ms[21 * 7] (host, may be
 * NULL) the best time of form f for class c at ms[c * 7 + f] (-1 where not
 * run).  Synchronises the stream; uses the basis's own J/K work buffer. */
enum { MESS_FORM_AUTO = 0, MESS_FORM_LANE = 1, MESS_FORM_ROWS = 2, MESS_FORM_PLANE = 3, MESS_FORM_COOP = 4,
       MESS_FORM_WAVE = 5, MESS_FORM_FP64 = 6 };
int mess_kernel_form(int32_t prec, int32_t cls, int32_t form, int32_t *active);
int mess_autotune(const mess_basis *basis, int32_t prec, double schwarz_tol, const double *D, int32_t reps,
                  int32_t *forms, double *ms, mess_stream stream);

/* Message for the last failing call on this thread ("" if none). */
const char *mess_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MESS_H */
