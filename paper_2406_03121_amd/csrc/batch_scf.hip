// Batched closed-shell SCF: many independent molecules advance together.
// Every matrix is packed block-diagonal (molecule m: n_m x n_m at offset
// moff[m]); the ERI classes of all molecules share one launch per class, and
// every dense step (Fock build, commutator, DIIS, orthonormal transform,
// purification, density) is one launch over all molecules.
//
// The step is the one of the single-molecule SCF (paper section 3, eq. 2):
// J, K <- D_k; F_k = H + J - K/2; E_k = 1/2 Tr[D_k (H + F_k)] + E_nuc;
// e_k = X^T (F D S - S D F) X; Pulay DIIS; D_{k+1} = 2 X P X^T with P the
// projector onto the n_occ lowest eigenvectors of X^T F X, by
// trace-correcting purification.  X is the Loewdin S^{-1/2} (Newton-Schulz).
//
// No decision in a step depends on the host: convergence, DIIS history and
// the end of purification are kept per molecule in device memory, and the
// purification runs a fixed number of rounds in which finished molecules do
// no work.  A step is therefore a fixed sequence of launches with fixed
// arguments, which is captured once into a HIP graph and replayed.
// A molecule whose energy change falls below the tolerance is frozen: its
// density stays the one that gave the converged energy.
//
// Divergence guard (per molecule, on unless opts.no_guard): the rule of the
// single-molecule SCF.  From iteration kGuardFrom on, an energy rise above
// kRiseTol counts against the molecule's stage, the second rise in a stage moves it to the next, a
// non-finite energy to the last; each change restarts its DIIS history
// (the molecule then uses only the entries pushed since: the history ring
// itself is shared).  Stage 2 mixes the next density half and half with the
// current one; stage 3 restarts the molecule from the core guess (damped).
#include <algorithm>
#include <cmath>
#include <vector>

#include "linalg.hpp"
#include "mess_internal.hpp"

namespace mess {

int jk_direct_half(mess_basis *B, const double *D, double *Gj, double *Gk, int prec, double tau, hipStream_t s);
int jk_stored(mess_basis *B, const double *D, double *Gj, double *Gk, int prec, double tau, hipStream_t s);

constexpr int kBMaxDiis = 16;
constexpr int kSp2Rounds = 100;  // purification rounds per step (finished molecules idle)
// Mixed-precision batches: the first kFarSteps Fock builds are complete FP32
// builds; then a complete FP64 build, FP32 builds of the density change added
// to it, and a complete FP64 rebuild after every kDeltaRun of those.
constexpr int kFarSteps = 2;
constexpr double kRiseTol = 1e-6;
constexpr int kRisesPerStage = 2;
constexpr int kGuardFrom = 12;  // rises count from this iteration on
constexpr double kDamp = 0.5;
constexpr int kDeltaRun = 8;
// Kinds of step (one captured graph each).
enum { kStepFull64 = 0, kStepFull64Open = 1, kStepFull32 = 2, kStepDelta32 = 3, kNumStepKinds = 4 };

struct MolScalars {
    double energy, e_new, de, resid;
    double emin, emax, trX, trX2, idem, scale;
    int sp2_iter, sp2_done, sp2_post, frozen;
    int sp2_fail;
    int stage, rises, hvalid;  // divergence guard; DIIS entries the molecule uses
    int fresh, restart, pad0, pad1;  // fresh: the next energy is compared with nothing
    double diis_c[kBMaxDiis + 1];
};

struct BatchState {
    int iter;
    int hcount, next_slot, last_slot;
    int hist[kBMaxDiis];
};

}  // namespace mess

struct mess_batch_scf {
    mess_basis *basis = nullptr;
    mess_scf_opts opts{};
    int nmol = 0, nmax = 0, nd = 0;
    int64_t packed = 0;
    bool use_graph = false;
    hipStream_t cap = nullptr;
    hipGraph_t graph[mess::kNumStepKinds] = {};
    hipGraphExec_t exec[mess::kNumStepKinds] = {};
    int host_iter = 0, since_full = 0;  // mixed precision: steps so far, dD builds since a complete FP64 build
    double *Dprev = nullptr, *dD = nullptr, *Gja = nullptr, *Gka = nullptr;  // mixed precision
    double *Dc = nullptr;  // core-Hamiltonian guess (divergence guard restarts)
    double *S = nullptr, *H = nullptr, *X = nullptr, *D = nullptr, *F = nullptr, *Fx = nullptr, *Gj = nullptr,
           *Gk = nullptr, *W1 = nullptr, *W2 = nullptr, *W3 = nullptr, *P = nullptr, *P2 = nullptr, *E = nullptr;
    double *Fh = nullptr, *Eh = nullptr, *Bm = nullptr;
    double *enuc = nullptr, *nocc = nullptr;
    mess::MolScalars *ms = nullptr;
    mess::BatchState *bs = nullptr;
};

namespace mess {

// Per-molecule loops: grid (chunks, molecules); blockIdx.y strides over
// molecules, x over the molecule's n^2 elements.
#define MOL_LOOP_BEGIN                                                     \
    for (int m = blockIdx.y; m < nmol; m += gridDim.y) {                   \
        const int n = nb[m];                                               \
        const int64_t o = moff[m], nn = (int64_t)n * n;                    \
        for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < nn; \
             idx += (int64_t)gridDim.x * blockDim.x) {
#define MOL_LOOP_END \
    }                \
    }

__device__ __forceinline__ double block_sum256(double v, double *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double block_max256(double v, double *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + st]);
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// F = H + (Gj + Gj^T) - 1/2 (Gk + Gk^T) and e_new = 1/2 sum D .* (H + F) + E_nuc
// (one block per molecule; frozen molecules are skipped).
__global__ void __launch_bounds__(256) k_bfock(int nmol, const int64_t *__restrict__ moff, const int *__restrict__ nb,
                                               const double *__restrict__ H, const double *__restrict__ Gj,
                                               const double *__restrict__ Gk, const double *__restrict__ D,
                                               const double *__restrict__ enuc, double *__restrict__ F,
                                               MolScalars *__restrict__ ms) {
    __shared__ double red[256];
    for (int m = blockIdx.x; m < nmol; m += gridDim.x) {
        if (ms[m].frozen) continue;
        const int n = nb[m];
        const int64_t o = moff[m], nn = (int64_t)n * n;
        double acc = 0.0;
        for (int64_t idx = threadIdx.x; idx < nn; idx += 256) {
            const int i = (int)(idx / n), j = (int)(idx % n);
            const int64_t t = o + (int64_t)j * n + i;
            const double f = H[o + idx] + (Gj[o + idx] + Gj[t]) - 0.5 * (Gk[o + idx] + Gk[t]);
            F[o + idx] = f;
            acc += D[o + idx] * (H[o + idx] + f);
        }
        const double tot = block_sum256(acc, red);
        if (threadIdx.x == 0) ms[m].e_new = 0.5 * tot + enuc[m];
    }
}

// C = Mx - Mx^T per block
__global__ void k_bantisym(int nmol, const int64_t *__restrict__ moff, const int *__restrict__ nb,
                           const double *__restrict__ Mx, double *__restrict__ C) {
    MOL_LOOP_BEGIN
    const int i = (int)(idx / n), j = (int)(idx % n);
    C[o + idx] = Mx[o + idx] - Mx[o + (int64_t)j * n + i];
    MOL_LOOP_END
}

// resid = max |e| per molecule (frozen molecules keep theirs)
__global__ void __launch_bounds__(256) k_bmaxabs(int nmol, const int64_t *__restrict__ moff,
                                                 const int *__restrict__ nb, const double *__restrict__ e,
                                                 MolScalars *__restrict__ ms) {
    __shared__ double red[256];
    for (int m = blockIdx.x; m < nmol; m += gridDim.x) {
        if (ms[m].frozen) continue;
        const int64_t o = moff[m], nn = (int64_t)nb[m] * nb[m];
        double v = 0.0;
        for (int64_t i = threadIdx.x; i < nn; i += 256) v = fmax(v, fabs(e[o + i]));
        v = block_max256(v, red);
        if (threadIdx.x == 0) ms[m].resid = v;
    }
}

// Energy bookkeeping, convergence and the divergence guard; one thread per
// molecule.  nd: DIIS history length (0: none).
__global__ void k_bconv(int nmol, double tol, int guard, int nd, const BatchState *__restrict__ bs,
                        MolScalars *__restrict__ ms) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= nmol || ms[m].frozen) return;
    MolScalars &q = ms[m];
    const bool have_prev = bs->iter > 0 && !q.fresh;
    q.fresh = 0;
    q.hvalid = min(q.hvalid + 1, nd);  // this step's entry
    const double e = q.e_new;
    if (!isfinite(e)) {
        if (guard && q.stage < 3) {  // straight to the restart; the energy field keeps its last value
            q.stage = 3;
            q.rises = 0;
            q.restart = 1;
            q.de = 0.0;
        } else {  // nothing left to try: frozen with the non-finite energy
            q.energy = e;
            q.de = 0.0;
            q.frozen = 1;
        }
        return;
    }
    const double de = have_prev ? e - q.energy : 0.0;
    q.energy = e;
    q.de = de;
    if (have_prev && fabs(de) < tol) {
        q.frozen = 1;
        return;
    }
    if (guard && have_prev && bs->iter >= kGuardFrom && de > kRiseTol && ++q.rises >= kRisesPerStage &&
        q.stage < 3) {
        q.stage += 1;
        q.rises = 0;
        q.hvalid = min(1, nd);
        if (q.stage == 3) q.restart = 1;
    }
}

// DIIS history: F and e of this step into slot next_slot.
__global__ void k_bdiis_push(int nmol, const int64_t *__restrict__ moff, const int *__restrict__ nb, int64_t packed,
                             const BatchState *__restrict__ bs, const double *__restrict__ F,
                             const double *__restrict__ e, double *__restrict__ Fh, double *__restrict__ Eh) {
    const int64_t so = (int64_t)bs->next_slot * packed;
    MOL_LOOP_BEGIN
    Fh[so + o + idx] = F[o + idx];
    Eh[so + o + idx] = e[o + idx];
    MOL_LOOP_END
}

__global__ void k_bdiis_book(int nd, BatchState *__restrict__ bs) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int slot = bs->next_slot;
    if (bs->hcount == nd) {
        for (int i = 1; i < nd; ++i) bs->hist[i - 1] = bs->hist[i];
        bs->hcount -= 1;
    }
    bs->hist[bs->hcount++] = slot;
    bs->last_slot = slot;
    bs->next_slot = (slot + 1) % nd;
}

// Bm[m][last][k] = Bm[m][k][last] = <E_last, E_k> over molecule m's block;
// grid (kBMaxDiis, molecules).
__global__ void __launch_bounds__(256) k_bdiis_dots(int nmol, const int64_t *__restrict__ moff,
                                                    const int *__restrict__ nb, int64_t packed,
                                                    const BatchState *__restrict__ bs, const double *__restrict__ Eh,
                                                    const MolScalars *__restrict__ ms, double *__restrict__ Bm) {
    __shared__ double red[256];
    const int h = blockIdx.x;
    if (h >= bs->hcount) return;
    const int slot = bs->last_slot, k = bs->hist[h];
    for (int m = blockIdx.y; m < nmol; m += gridDim.y) {
        if (ms[m].frozen) continue;
        const int64_t o = moff[m], nn = (int64_t)nb[m] * nb[m];
        const double *a = Eh + (int64_t)slot * packed + o, *b = Eh + (int64_t)k * packed + o;
        double acc = 0.0;
        for (int64_t i = threadIdx.x; i < nn; i += 256) acc += a[i] * b[i];
        acc = block_sum256(acc, red);
        if (threadIdx.x == 0) {
            double *Bmm = Bm + (int64_t)m * kBMaxDiis * kBMaxDiis;
            Bmm[slot * kBMaxDiis + k] = acc;
            Bmm[k * kBMaxDiis + slot] = acc;
        }
    }
}

// Coefficients: solve [[B, -1], [-1^T, 0]] [c; lambda] = [0; -1] by Gaussian
// elimination with partial pivoting (one thread per molecule); with a single
// history entry c = 1.
__global__ void k_bdiis_solve(int nmol, const BatchState *__restrict__ bs, const double *__restrict__ Bm,
                              MolScalars *__restrict__ ms) {
    const int mol = blockIdx.x * blockDim.x + threadIdx.x;
    if (mol >= nmol || ms[mol].frozen) return;
    // the molecule's own (most recent) entries of the shared history
    const int m = min(bs->hcount, ms[mol].hvalid), h0 = bs->hcount - m;
    if (m < 2) {
        ms[mol].diis_c[0] = 1.0;
        return;
    }
    const double *Bmm = Bm + (int64_t)mol * kBMaxDiis * kBMaxDiis;
    double A[kBMaxDiis + 1][kBMaxDiis + 2];
    const int n = m + 1;
    for (int i = 0; i < m; ++i) {
        for (int j = 0; j < m; ++j) A[i][j] = Bmm[bs->hist[h0 + i] * kBMaxDiis + bs->hist[h0 + j]];
        A[i][m] = -1.0;
        A[i][n] = 0.0;
    }
    for (int j = 0; j < m; ++j) A[m][j] = -1.0;
    A[m][m] = 0.0;
    A[m][n] = -1.0;
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
        if (piv != col)
            for (int c = 0; c <= n; ++c) {
                const double t = A[col][c];
                A[col][c] = A[piv][c];
                A[piv][c] = t;
            }
        const double d = A[col][col];
        for (int r = col + 1; r < n; ++r) {
            const double f = d != 0.0 ? A[r][col] / d : 0.0;
            for (int c = col; c <= n; ++c) A[r][c] -= f * A[col][c];
        }
    }
    double x[kBMaxDiis + 1];
    for (int r = n - 1; r >= 0; --r) {
        double s = A[r][n];
        for (int c = r + 1; c < n; ++c) s -= A[r][c] * x[c];
        x[r] = A[r][r] != 0.0 ? s / A[r][r] : 0.0;
    }
    for (int i = 0; i < m; ++i) ms[mol].diis_c[i] = x[i];
}

// Fx = sum_i c_i Fh[hist_i] per molecule
__global__ void k_bdiis_combine(int nmol, const int64_t *__restrict__ moff, const int *__restrict__ nb, int64_t packed,
                                const BatchState *__restrict__ bs, const double *__restrict__ Fh,
                                const MolScalars *__restrict__ ms, double *__restrict__ Fx) {
    const int hc = bs->hcount;
    MOL_LOOP_BEGIN
    const int k = max(1, min(hc, ms[m].hvalid)), h0 = hc - k;
    double v = 0.0;
    for (int i = 0; i < k; ++i) v += ms[m].diis_c[i] * Fh[(int64_t)bs->hist[h0 + i] * packed + o + idx];
    Fx[o + idx] = v;
    MOL_LOOP_END
}

// Gershgorin bounds of each block -> emin, emax; resets the purification
// state (frozen molecules are marked finished).  One block per molecule.
__global__ void __launch_bounds__(256) k_bgershgorin(int nmol, const int64_t *__restrict__ moff,
                                                     const int *__restrict__ nb, const double *__restrict__ A,
                                                     MolScalars *__restrict__ ms) {
    __shared__ double red[256];
    for (int m = blockIdx.x; m < nmol; m += gridDim.x) {
        const int n = nb[m];
        const double *Am = A + moff[m];
        double l = 1e300, h = -1e300;
        for (int i = threadIdx.x; i < n; i += 256) {
            double r = 0.0;
            for (int j = 0; j < n; ++j)
                if (j != i) r += fabs(Am[(int64_t)i * n + j]);
            const double d = Am[(int64_t)i * n + i];
            l = fmin(l, d - r);
            h = fmax(h, d + r);
        }
        l = -block_max256(-l, red);
        h = block_max256(h, red);
        if (threadIdx.x == 0) {
            ms[m].emin = l;
            ms[m].emax = h > l ? h : l + 1.0;
            ms[m].sp2_iter = 0;
            ms[m].sp2_done = ms[m].frozen;
            ms[m].sp2_post = 0;
            ms[m].sp2_fail = 0;
        }
    }
}

// X0 = (e_max I - F') / (e_max - e_min)
__global__ void k_bsp2_init(int nmol, const int64_t *__restrict__ moff, const int *__restrict__ nb,
                            const double *__restrict__ Fp, const MolScalars *__restrict__ ms, double *__restrict__ X) {
    MOL_LOOP_BEGIN
    const double emax = ms[m].emax, inv = 1.0 / (ms[m].emax - ms[m].emin);
    const int i = (int)(idx / n), j = (int)(idx % n);
    X[o + idx] = ((i == j ? emax : 0.0) - Fp[o + idx]) * inv;
    MOL_LOOP_END
}

__global__ void __launch_bounds__(256) k_bsp2_traces(int nmol, const int64_t *__restrict__ moff,
                                                     const int *__restrict__ nb, const double *__restrict__ X,
                                                     const double *__restrict__ X2, MolScalars *__restrict__ ms) {
    __shared__ double red[256];
    for (int m = blockIdx.x; m < nmol; m += gridDim.x) {
        if (ms[m].sp2_done) continue;
        const int n = nb[m];
        const int64_t o = moff[m];
        double s1 = 0.0, s2 = 0.0;
        for (int i = threadIdx.x; i < n; i += 256) {
            s1 += X[o + (int64_t)i * n + i];
            s2 += X2[o + (int64_t)i * n + i];
        }
        s1 = block_sum256(s1, red);
        s2 = block_sum256(s2, red);
        if (threadIdx.x == 0) {
            ms[m].trX = s1;
            ms[m].trX2 = s2;
            ms[m].idem = s1 - s2;
        }
    }
}

__global__ void k_bsp2_update(int nmol, const int64_t *__restrict__ moff, const int *__restrict__ nb,
                              const double *__restrict__ nocc, double *__restrict__ X, const double *__restrict__ X2,
                              const MolScalars *__restrict__ ms) {
    for (int m = blockIdx.y; m < nmol; m += gridDim.y) {
        if (ms[m].sp2_done) continue;
        const int n = nb[m];
        const int64_t o = moff[m], nn = (int64_t)n * n;
        const double t1 = ms[m].trX, t2 = ms[m].trX2, no = nocc[m];
        const bool square = fabs(t2 - no) < fabs(2.0 * t1 - t2 - no);
        for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < nn;
             idx += (int64_t)gridDim.x * blockDim.x)
            X[o + idx] = square ? X2[o + idx] : 2.0 * X[o + idx] - X2[o + idx];
    }
}

__global__ void k_bsp2_book(int nmol, MolScalars *__restrict__ ms, int last) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= nmol || ms[m].sp2_done) return;
    ms[m].sp2_iter += 1;
    // once idempotent to 1e-10, two more quadratic steps reach rounding level
    if (ms[m].sp2_post > 0 || fabs(ms[m].idem) < 1e-10) ms[m].sp2_post += 1;
    if (ms[m].sp2_post >= 3) ms[m].sp2_done = 1;
    else if (last) ms[m].sp2_fail = 1;
}

// Next density of every molecule that is not frozen: Dn; from guard stage 2
// (1 - kDamp) Dn + kDamp D; the core guess Dc for a molecule restarting.
__global__ void k_bnext_density(int nmol, const int64_t *__restrict__ moff, const int *__restrict__ nb,
                                const MolScalars *__restrict__ ms, const double *__restrict__ Dn,
                                const double *__restrict__ Dc, double *__restrict__ D) {
    for (int m = blockIdx.y; m < nmol; m += gridDim.y) {
        if (ms[m].frozen) continue;
        const int n = nb[m], mode = ms[m].restart ? 2 : ms[m].stage >= 2 ? 1 : 0;
        const int64_t o = moff[m], nn = (int64_t)n * n;
        for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < nn;
             idx += (int64_t)gridDim.x * blockDim.x) {
            const double dn = Dn[o + idx];
            D[o + idx] = mode == 0 ? dn : mode == 1 ? (1.0 - kDamp) * dn + kDamp * D[o + idx] : Dc[o + idx];
        }
    }
}

// After a restart: no DIIS entries, the next energy compared with nothing,
// and the discarded purification's outcome forgotten.
__global__ void k_brestart_book(int nmol, MolScalars *__restrict__ ms) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= nmol || !ms[m].restart) return;
    ms[m].restart = 0;
    ms[m].hvalid = 0;
    ms[m].fresh = 1;
    ms[m].sp2_fail = 0;
}

__global__ void k_bstep_end(BatchState *__restrict__ bs) {
    if (threadIdx.x == 0 && blockIdx.x == 0) bs->iter += 1;
}

// out = a I + b Z per block
__global__ void k_bident_plus(int nmol, const int64_t *__restrict__ moff, const int *__restrict__ nb, double a,
                              double b, const double *__restrict__ Z, double *__restrict__ out) {
    MOL_LOOP_BEGIN
    const int i = (int)(idx / n), j = (int)(idx % n);
    out[o + idx] = (i == j ? a : 0.0) + b * Z[o + idx];
    MOL_LOOP_END
}

// out = src / scale_m (src != NULL) or the identity; scale_m = ms[m].scale
__global__ void k_bscaled(int nmol, const int64_t *__restrict__ moff, const int *__restrict__ nb,
                          const MolScalars *__restrict__ ms, int use_sqrt, const double *__restrict__ src,
                          double *__restrict__ out) {
    MOL_LOOP_BEGIN
    const double c = use_sqrt ? sqrt(ms[m].scale) : ms[m].scale;
    out[o + idx] = src ? src[o + idx] / c : ((idx / n == idx % n) ? 1.0 : 0.0);
    MOL_LOOP_END
}

// resid = max |A - I| per block; with inf_norm, trX = max row sum of |A|.
__global__ void __launch_bounds__(256) k_bnorms(int nmol, const int64_t *__restrict__ moff, const int *__restrict__ nb,
                                                const double *__restrict__ A, int inf_norm,
                                                MolScalars *__restrict__ ms) {
    __shared__ double red[256];
    for (int m = blockIdx.x; m < nmol; m += gridDim.x) {
        const int n = nb[m];
        const double *Am = A + moff[m];
        double v = 0.0;
        if (inf_norm) {
            for (int i = threadIdx.x; i < n; i += 256) {
                double r = 0.0;
                for (int j = 0; j < n; ++j) r += fabs(Am[(int64_t)i * n + j]);
                v = fmax(v, r);
            }
        } else {
            for (int64_t i = threadIdx.x; i < (int64_t)n * n; i += 256)
                v = fmax(v, fabs(Am[i] - ((i / n == i % n) ? 1.0 : 0.0)));
        }
        v = block_max256(v, red);
        if (threadIdx.x == 0) {
            if (inf_norm) ms[m].trX = v;
            else ms[m].resid = v;
        }
    }
}

__global__ void k_bset_scale_emax(int nmol, MolScalars *__restrict__ ms) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < nmol) ms[m].scale = ms[m].emax;
}

__global__ void k_bcopy(int64_t n, const double *__restrict__ src, double *__restrict__ dst) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

#undef MOL_LOOP_BEGIN
#undef MOL_LOOP_END

// ------------------------------------------------------------------ host

struct BLaunch {
    int nmol, nmax;
    const int64_t *moff;
    const int *nb;
    dim3 ew, per_mol, per_thread;  // elementwise grid, block-per-molecule grid, thread-per-molecule grid
};

static BLaunch blaunch(const mess_batch_scf *st) {
    const mess_basis *B = st->basis;
    BLaunch L;
    L.nmol = st->nmol;
    L.nmax = st->nmax;
    L.moff = B->d_mol_moff;
    L.nb = B->d_mol_nbf;
    const int64_t nn = (int64_t)st->nmax * st->nmax;
    int64_t cx = (nn + 255) / 256;
    if (cx > 64) cx = 64;
    L.ew = dim3((unsigned)std::max<int64_t>(cx, 1), (unsigned)std::min(st->nmol, 65535));
    L.per_mol = dim3((unsigned)std::min(st->nmol, 65535));
    L.per_thread = dim3((unsigned)((st->nmol + 63) / 64));
    return L;
}

static int bgemm(const mess_batch_scf *st, hipStream_t s, bool ta, bool tb, double alpha, const double *A,
                 const double *Bm, double beta, double *C) {
    return gemm_blocks(s, ta, tb, st->nmol, st->nmax, st->basis->d_mol_moff, st->basis->d_mol_nbf, alpha, A, Bm,
                       beta, C);
}

// Fp = X^T F X per block (W3 holds X^T F)
static int to_orthonormal(mess_batch_scf *st, const double *F, double *Fp, hipStream_t s) {
    MESS_TRY(bgemm(st, s, true, false, 1.0, st->X, F, 0.0, st->W3));
    MESS_TRY(bgemm(st, s, false, false, 1.0, st->W3, st->X, 0.0, Fp));
    return MESS_OK;
}

// P <- projector of Fp (fixed number of rounds); Dn = 2 X P X^T
static int purify_density(mess_batch_scf *st, const double *Fp, double *Dn, hipStream_t s) {
    const BLaunch L = blaunch(st);
    hipLaunchKernelGGL(k_bgershgorin, L.per_mol, dim3(256), 0, s, L.nmol, L.moff, L.nb, Fp, st->ms);
    hipLaunchKernelGGL(k_bsp2_init, L.ew, dim3(256), 0, s, L.nmol, L.moff, L.nb, Fp, st->ms, st->P);
    MESS_LAUNCH_CHECK();
    for (int r = 0; r < kSp2Rounds; ++r) {
        MESS_TRY(bgemm(st, s, false, false, 1.0, st->P, st->P, 0.0, st->P2));
        hipLaunchKernelGGL(k_bsp2_traces, L.per_mol, dim3(256), 0, s, L.nmol, L.moff, L.nb, st->P, st->P2, st->ms);
        hipLaunchKernelGGL(k_bsp2_update, L.ew, dim3(256), 0, s, L.nmol, L.moff, L.nb, st->nocc, st->P, st->P2,
                           st->ms);
        hipLaunchKernelGGL(k_bsp2_book, L.per_thread, dim3(64), 0, s, L.nmol, st->ms, r == kSp2Rounds - 1 ? 1 : 0);
    }
    MESS_LAUNCH_CHECK();
    MESS_TRY(bgemm(st, s, false, false, 1.0, st->X, st->P, 0.0, st->W1));
    MESS_TRY(bgemm(st, s, false, true, 2.0, st->W1, st->X, 0.0, Dn));
    return MESS_OK;
}

static int batch_jk(mess_batch_scf *st, const double *D, double *Gj, double *Gk, int prec, hipStream_t s) {
    if (st->opts.jk_mode == MESS_JK_DIRECT)
        return jk_direct_half(st->basis, D, Gj, Gk, prec, st->opts.schwarz_tol, s);
    return jk_stored(st->basis, D, Gj, Gk, prec, st->opts.schwarz_tol, s);
}

static int enqueue_step(mess_batch_scf *st, hipStream_t s, int kind) {
    const BLaunch L = blaunch(st);
    const double *Gjf = st->Gj, *Gkf = st->Gk;
    bool may_converge = kind == kStepFull64 || kind == kStepDelta32;
    if (st->opts.prec != MESS_FP32) {
        MESS_TRY(batch_jk(st, st->D, st->Gj, st->Gk, MESS_FP64, s));
        may_converge = true;
    } else {
        // mixed precision: the running half-matrices Gja/Gka
        if (kind == kStepDelta32) {
            MESS_TRY(axpby(s, st->packed, 1.0, st->D, -1.0, st->Dprev, st->dD));
            MESS_TRY(batch_jk(st, st->dD, st->Gj, st->Gk, MESS_FP32, s));
            MESS_TRY(axpby(s, st->packed, 1.0, st->Gja, 1.0, st->Gj, st->Gja));
            MESS_TRY(axpby(s, st->packed, 1.0, st->Gka, 1.0, st->Gk, st->Gka));
        } else {
            MESS_TRY(batch_jk(st, st->D, st->Gja, st->Gka, kind == kStepFull32 ? MESS_FP32 : MESS_FP64, s));
        }
        hipLaunchKernelGGL(k_bcopy, dim3((unsigned)std::min<int64_t>((st->packed + 255) / 256, 65536)), dim3(256), 0,
                           s, st->packed, st->D, st->Dprev);
        Gjf = st->Gja;
        Gkf = st->Gka;
    }
    hipLaunchKernelGGL(k_bfock, L.per_mol, dim3(256), 0, s, L.nmol, L.moff, L.nb, st->H, Gjf, Gkf, st->D,
                       st->enuc, st->F, st->ms);
    MESS_LAUNCH_CHECK();
    // e = X^T (F D S - S D F) X
    MESS_TRY(bgemm(st, s, false, false, 1.0, st->F, st->D, 0.0, st->W1));
    MESS_TRY(bgemm(st, s, false, false, 1.0, st->W1, st->S, 0.0, st->W2));
    hipLaunchKernelGGL(k_bantisym, L.ew, dim3(256), 0, s, L.nmol, L.moff, L.nb, st->W2, st->W1);
    MESS_LAUNCH_CHECK();
    MESS_TRY(bgemm(st, s, true, false, 1.0, st->X, st->W1, 0.0, st->W3));
    MESS_TRY(bgemm(st, s, false, false, 1.0, st->W3, st->X, 0.0, st->E));
    hipLaunchKernelGGL(k_bmaxabs, L.per_mol, dim3(256), 0, s, L.nmol, L.moff, L.nb, st->E, st->ms);
    // only energies on FP64-anchored J/K following another such energy may
    // freeze a molecule (a negative tolerance freezes none)
    hipLaunchKernelGGL(k_bconv, L.per_thread, dim3(64), 0, s, L.nmol, may_converge ? st->opts.conv_tol : -1.0,
                       st->opts.no_guard ? 0 : 1, st->nd, st->bs, st->ms);
    MESS_LAUNCH_CHECK();
    const double *Fuse = st->F;
    if (st->nd > 0) {
        hipLaunchKernelGGL(k_bdiis_push, L.ew, dim3(256), 0, s, L.nmol, L.moff, L.nb, st->packed, st->bs, st->F,
                           st->E, st->Fh, st->Eh);
        hipLaunchKernelGGL(k_bdiis_book, dim3(1), dim3(64), 0, s, st->nd, st->bs);
        hipLaunchKernelGGL(k_bdiis_dots, dim3(kBMaxDiis, std::min(L.nmol, 65535)), dim3(256), 0, s, L.nmol, L.moff,
                           L.nb, st->packed, st->bs, st->Eh, st->ms, st->Bm);
        hipLaunchKernelGGL(k_bdiis_solve, L.per_thread, dim3(64), 0, s, L.nmol, st->bs, st->Bm, st->ms);
        hipLaunchKernelGGL(k_bdiis_combine, L.ew, dim3(256), 0, s, L.nmol, L.moff, L.nb, st->packed, st->bs, st->Fh,
                           st->ms, st->Fx);
        MESS_LAUNCH_CHECK();
        Fuse = st->Fx;
    }
    MESS_TRY(to_orthonormal(st, Fuse, st->W2, s));
    MESS_TRY(purify_density(st, st->W2, st->W2, s));  // Fp is consumed before Dn is written
    hipLaunchKernelGGL(k_bnext_density, L.ew, dim3(256), 0, s, L.nmol, L.moff, L.nb, st->ms, st->W2, st->Dc, st->D);
    hipLaunchKernelGGL(k_brestart_book, L.per_thread, dim3(64), 0, s, L.nmol, st->ms);
    hipLaunchKernelGGL(k_bstep_end, dim3(1), dim3(64), 0, s, st->bs);
    MESS_LAUNCH_CHECK();
    return MESS_OK;
}

static void free_batch(mess_batch_scf *st) {
    if (!st) return;
    for (int k = 0; k < kNumStepKinds; ++k) {
        if (st->exec[k]) hipGraphExecDestroy(st->exec[k]);
        if (st->graph[k]) hipGraphDestroy(st->graph[k]);
    }
    if (st->cap) hipStreamDestroy(st->cap);
    for (double *p : {st->S, st->H, st->X, st->D, st->F, st->Fx, st->Gj, st->Gk, st->W1, st->W2, st->W3, st->P,
                      st->P2, st->E, st->Fh, st->Eh, st->Bm, st->enuc, st->nocc, st->Dprev, st->dD, st->Gja, st->Gka,
                      st->Dc})
        hipFree(p);
    hipFree(st->ms);
    hipFree(st->bs);
    delete st;
}

// Loewdin X = S^{-1/2} per block by the coupled Newton-Schulz iteration on
// A = S / c_m (c_m: Gershgorin bound of block m): T = (3 I - Z Y)/2,
// Y <- Y T, Z <- T Z from Y = A, Z = I.  Fails (E_NUMERIC) for a molecule
// whose smallest overlap eigenvalue cannot be bounded above 1e-6.
static int batch_lowdin(mess_batch_scf *st, hipStream_t s) {
    const BLaunch L = blaunch(st);
    hipLaunchKernelGGL(k_bgershgorin, L.per_mol, dim3(256), 0, s, L.nmol, L.moff, L.nb, st->S, st->ms);
    hipLaunchKernelGGL(k_bset_scale_emax, L.per_thread, dim3(64), 0, s, L.nmol, st->ms);
    double *Y = st->Gj, *Z = st->Gk, *T = st->F, *tmp = st->Fx;
    hipLaunchKernelGGL(k_bscaled, L.ew, dim3(256), 0, s, L.nmol, L.moff, L.nb, st->ms, 0, st->S, Y);
    hipLaunchKernelGGL(k_bscaled, L.ew, dim3(256), 0, s, L.nmol, L.moff, L.nb, st->ms, 0, nullptr, Z);
    MESS_LAUNCH_CHECK();
    std::vector<MolScalars> h(st->nmol);
    bool conv = false;
    for (int it = 0; it < 80 && !conv; ++it) {
        MESS_TRY(bgemm(st, s, false, false, 1.0, Z, Y, 0.0, tmp));
        if (it % 4 == 3) {
            hipLaunchKernelGGL(k_bnorms, L.per_mol, dim3(256), 0, s, L.nmol, L.moff, L.nb, tmp, 0, st->ms);
            MESS_HIP(hipMemcpyAsync(h.data(), st->ms, sizeof(MolScalars) * st->nmol, hipMemcpyDeviceToHost, s));
            MESS_HIP(hipStreamSynchronize(s));
            conv = true;
            for (int m = 0; m < st->nmol; ++m) {
                if (!std::isfinite(h[m].resid)) {
                    set_error("mess_batch_scf_create: overlap orthogonalisation diverged for molecule %d", m);
                    return MESS_E_NUMERIC;
                }
                if (!(h[m].resid < 1e-14)) conv = false;
            }
        }
        hipLaunchKernelGGL(k_bident_plus, L.ew, dim3(256), 0, s, L.nmol, L.moff, L.nb, 1.5, -0.5, tmp, T);
        MESS_TRY(bgemm(st, s, false, false, 1.0, Y, T, 0.0, tmp));
        std::swap(Y, tmp);
        MESS_TRY(bgemm(st, s, false, false, 1.0, T, Z, 0.0, tmp));
        std::swap(Z, tmp);
    }
    if (!conv) {
        set_error("mess_batch_scf_create: overlap orthogonalisation did not converge");
        return MESS_E_NUMERIC;
    }
    hipLaunchKernelGGL(k_bscaled, L.ew, dim3(256), 0, s, L.nmol, L.moff, L.nb, st->ms, 1, Z, st->X);
    MESS_LAUNCH_CHECK();
    MESS_TRY(bgemm(st, s, false, false, 1.0, st->X, st->X, 0.0, tmp));
    hipLaunchKernelGGL(k_bnorms, L.per_mol, dim3(256), 0, s, L.nmol, L.moff, L.nb, tmp, 1, st->ms);
    MESS_HIP(hipMemcpyAsync(h.data(), st->ms, sizeof(MolScalars) * st->nmol, hipMemcpyDeviceToHost, s));
    MESS_HIP(hipStreamSynchronize(s));
    for (int m = 0; m < st->nmol; ++m)
        if (!(std::isfinite(h[m].trX) && h[m].trX > 0.0 && 1.0 / h[m].trX > 1e-6)) {
            set_error("mess_batch_scf_create: overlap of molecule %d may be near-singular (batched SCF keeps all "
                      "functions); run it alone with mess_scf_create",
                      m);
            return MESS_E_NUMERIC;
        }
    // two Newton steps X <- X (3 I - X^T S X) / 2
    for (int k = 0; k < 2; ++k) {
        MESS_TRY(bgemm(st, s, false, false, 1.0, st->S, st->X, 0.0, st->W1));
        MESS_TRY(bgemm(st, s, true, false, 1.0, st->X, st->W1, 0.0, st->P));
        hipLaunchKernelGGL(k_bident_plus, L.ew, dim3(256), 0, s, L.nmol, L.moff, L.nb, 1.5, -0.5, st->P, st->P2);
        MESS_TRY(bgemm(st, s, false, false, 1.0, st->X, st->P2, 0.0, st->W1));
        hipLaunchKernelGGL(k_bcopy, dim3(1024), dim3(256), 0, s, st->packed, st->W1, st->X);
        MESS_LAUNCH_CHECK();
    }
    return MESS_OK;
}

// ortho_only: one-electron matrices and X only (no density, no J/K set-up).
static int batch_create_impl(mess_batch_scf *st, const double *D0, bool ortho_only = false) {
    mess_basis *B = st->basis;
    st->nmol = B->n_mol;
    st->nmax = B->nbf_max;
    st->packed = B->packed;
    st->nd = std::max(0, std::min(st->opts.diis_size, kBMaxDiis));
    hipStream_t s = nullptr;
    const size_t pk = (size_t)std::max<int64_t>(B->packed, 16);
    for (double **p : {&st->S, &st->H, &st->X, &st->D, &st->F, &st->Fx, &st->Gj, &st->Gk, &st->W1, &st->W2, &st->W3,
                       &st->P, &st->P2, &st->E})
        MESS_HIP(hipMalloc(p, sizeof(double) * pk));
    const int nd1 = std::max(1, st->nd);
    MESS_HIP(hipMalloc(&st->Fh, sizeof(double) * pk * nd1));
    MESS_HIP(hipMalloc(&st->Eh, sizeof(double) * pk * nd1));
    MESS_HIP(hipMalloc(&st->Bm, sizeof(double) * kBMaxDiis * kBMaxDiis * st->nmol));
    if (st->opts.prec == MESS_FP32)
        for (double **p : {&st->Dprev, &st->dD, &st->Gja, &st->Gka}) MESS_HIP(hipMalloc(p, sizeof(double) * pk));
    MESS_HIP(hipMalloc(&st->enuc, sizeof(double) * st->nmol));
    MESS_HIP(hipMalloc(&st->nocc, sizeof(double) * st->nmol));
    MESS_HIP(hipMalloc(&st->ms, sizeof(MolScalars) * st->nmol));
    MESS_HIP(hipMalloc(&st->bs, sizeof(BatchState)));
    MESS_HIP(hipMemset(st->ms, 0, sizeof(MolScalars) * st->nmol));
    MESS_HIP(hipMemset(st->bs, 0, sizeof(BatchState)));
    {
        std::vector<double> no(st->nmol);
        for (int m = 0; m < st->nmol; ++m) no[m] = B->mol_nocc[m];
        MESS_HIP(hipMemcpy(st->enuc, B->mol_enuc.data(), sizeof(double) * st->nmol, hipMemcpyHostToDevice));
        MESS_HIP(hipMemcpy(st->nocc, no.data(), sizeof(double) * st->nmol, hipMemcpyHostToDevice));
    }
    MESS_TRY(mess_one_electron(B, st->S, st->W1, st->W2, s));
    MESS_TRY(axpby(s, B->packed, 1.0, st->W1, 1.0, st->W2, st->H));
    MESS_TRY(batch_lowdin(st, s));
    if (ortho_only) {
        MESS_HIP(hipStreamSynchronize(s));
        MESS_HIP(hipMemset(st->ms, 0, sizeof(MolScalars) * st->nmol));
        return MESS_OK;
    }
    // core guess: the initial density unless D0 is given, and the guard's
    // restart point
    if (!D0 || !st->opts.no_guard) {
        MESS_TRY(to_orthonormal(st, st->H, st->W2, s));
        MESS_TRY(purify_density(st, st->W2, st->W2, s));
    }
    if (!st->opts.no_guard) {
        MESS_HIP(hipMalloc(&st->Dc, sizeof(double) * pk));
        MESS_HIP(hipMemcpyAsync(st->Dc, st->W2, sizeof(double) * B->packed, hipMemcpyDeviceToDevice, s));
    }
    MESS_HIP(hipMemcpyAsync(st->D, D0 ? D0 : st->W2, sizeof(double) * B->packed, hipMemcpyDeviceToDevice, s));
    // the purification state of the guess is not a step's: reset it
    MESS_HIP(hipMemsetAsync(st->ms, 0, sizeof(MolScalars) * st->nmol, s));
    // work lists (and the stored integrals, in every precision a step uses)
    // are built here, so that a step allocates nothing and can be captured
    MESS_TRY(batch_jk(st, st->D, st->Gj, st->Gk, MESS_FP64, s));
    if (st->opts.prec == MESS_FP32) MESS_TRY(batch_jk(st, st->D, st->Gj, st->Gk, MESS_FP32, s));
    MESS_HIP(hipStreamSynchronize(s));
    if (st->use_graph) MESS_HIP(hipStreamCreateWithFlags(&st->cap, hipStreamNonBlocking));
    return MESS_OK;
}

// Natural-orbital projection: with X = S^-1/2 and S^1/2 = S X, the
// projector P onto the n_occ lowest eigenvectors of -S^1/2 D S^1/2 (the
// n_occ largest of S^1/2 D S^1/2) by the same purification as the SCF step;
// D <- 2 X P X.
static int project_impl(mess_batch_scf *st, double *D, hipStream_t s) {
    const BLaunch L = blaunch(st);
    MESS_TRY(bgemm(st, s, false, false, 1.0, st->S, st->X, 0.0, st->Gj));   // S^1/2
    MESS_TRY(bgemm(st, s, false, false, 1.0, st->Gj, D, 0.0, st->Gk));
    MESS_TRY(bgemm(st, s, false, false, 1.0, st->Gk, st->Gj, 0.0, st->W3));
    hipLaunchKernelGGL(k_bident_plus, L.ew, dim3(256), 0, s, L.nmol, L.moff, L.nb, 0.0, -1.0, st->W3, st->Fx);
    MESS_LAUNCH_CHECK();
    MESS_TRY(purify_density(st, st->Fx, D, s));
    return MESS_OK;
}

}  // namespace mess

using namespace mess;

extern "C" {

int mess_guess_project(const mess_basis *basis, double *D, mess_stream stream) {
    if (!basis || !D) {
        set_error("mess_guess_project: NULL argument");
        return MESS_E_ARG;
    }
    for (int m = 0; m < basis->n_mol; ++m)
        if (basis->mol_nelec[m] % 2) {
            set_error("mess_guess_project: molecule %d has an odd electron count", m);
            return MESS_E_UNSUPPORTED;
        }
    auto *st = new mess_batch_scf();
    st->basis = const_cast<mess_basis *>(basis);
    st->opts.diis_size = 0;
    int rc = batch_create_impl(st, nullptr, true);
    if (rc == MESS_OK) rc = project_impl(st, D, static_cast<hipStream_t>(stream));
    if (rc == MESS_OK && hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess) {
        set_error("mess_guess_project: device error");
        rc = MESS_E_DEVICE;
    }
    if (rc == MESS_OK) {
        std::vector<MolScalars> h(st->nmol);
        if (hipMemcpy(h.data(), st->ms, sizeof(MolScalars) * st->nmol, hipMemcpyDeviceToHost) != hipSuccess) {
            rc = MESS_E_DEVICE;
        } else {
            for (int m = 0; m < st->nmol; ++m)
                if (h[m].sp2_fail) {
                    set_error("mess_guess_project: purification of molecule %d did not finish", m);
                    rc = MESS_E_NUMERIC;
                    break;
                }
        }
    }
    free_batch(st);
    return rc;
}

int mess_guess_judge(const mess_basis *basis, const mess_scf_opts *opts, double *D0, int32_t *used,
                     mess_stream stream) {
    if (!basis || !opts || !D0) {
        set_error("mess_guess_judge: NULL argument");
        return MESS_E_ARG;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    MESS_HIP(hipStreamSynchronize(s));
    mess_batch_scf *a = nullptr, *b = nullptr;
    MESS_TRY(mess_batch_scf_create(basis, opts, D0, 0, &a));
    int rc = mess_batch_scf_create(basis, opts, nullptr, 0, &b);
    double *Dcore = nullptr;
    std::vector<double> ra(basis->n_mol), rb(basis->n_mol);
    if (rc == MESS_OK && hipMalloc(&Dcore, sizeof(double) * std::max<int64_t>(basis->packed, 1)) != hipSuccess)
        rc = MESS_E_NOMEM;
    if (rc == MESS_OK && hipMemcpyAsync(Dcore, b->D, sizeof(double) * basis->packed, hipMemcpyDeviceToDevice, s) !=
                             hipSuccess)
        rc = MESS_E_DEVICE;
    if (rc == MESS_OK) rc = mess_batch_scf_step(a, s);
    if (rc == MESS_OK) rc = mess_batch_scf_step(b, s);
    if (rc == MESS_OK) rc = mess_batch_scf_status(a, nullptr, nullptr, ra.data(), nullptr, nullptr, s);
    if (rc == MESS_OK) rc = mess_batch_scf_status(b, nullptr, nullptr, rb.data(), nullptr, nullptr, s);
    if (rc == MESS_OK) {
        for (int m = 0; m < basis->n_mol && rc == MESS_OK; ++m) {
            const bool keep = ra[m] < rb[m];
            if (used) used[m] = keep ? 1 : 0;
            if (!keep &&
                hipMemcpyAsync(D0 + basis->mol_moff[m], Dcore + basis->mol_moff[m],
                               sizeof(double) * (size_t)basis->mol_nbf[m] * basis->mol_nbf[m],
                               hipMemcpyDeviceToDevice, s) != hipSuccess)
                rc = MESS_E_DEVICE;
        }
        if (rc == MESS_OK && hipStreamSynchronize(s) != hipSuccess) rc = MESS_E_DEVICE;
        if (rc == MESS_E_DEVICE) set_error("mess_guess_judge: device copy failed");
    }
    hipFree(Dcore);
    mess_batch_scf_destroy(a);
    mess_batch_scf_destroy(b);
    return rc;
}

int mess_batch_scf_create(const mess_basis *basis, const mess_scf_opts *opts, const double *D0, int32_t use_graph,
                          mess_batch_scf **out) {
    if (!basis || !opts || !out) {
        set_error("mess_batch_scf_create: NULL basis, options or output");
        return MESS_E_ARG;
    }
    *out = nullptr;
    for (int m = 0; m < basis->n_mol; ++m)
        if (basis->mol_nelec[m] % 2) {
            set_error("mess_batch_scf_create: molecule %d has %d electrons; only closed-shell systems are supported",
                      m, basis->mol_nelec[m]);
            return MESS_E_UNSUPPORTED;
        }
    if (opts->deterministic) {
        set_error("mess_batch_scf_create: the deterministic mode reads a host flag after every build; "
                  "run batches of it through mess_jk(MESS_JK_DETERMINISTIC) or single-molecule SCFs");
        return MESS_E_UNSUPPORTED;
    }
    if (opts->jk_mode != MESS_JK_DIRECT && opts->jk_mode != MESS_JK_STORED) {
        set_error("mess_batch_scf_create: unknown J/K mode %d", opts->jk_mode);
        return MESS_E_UNSUPPORTED;
    }
    if (opts->prec != MESS_FP64 && opts->prec != MESS_FP32) {
        set_error("mess_batch_scf_create: unknown precision %d", opts->prec);
        return MESS_E_UNSUPPORTED;
    }
    if (opts->xc != MESS_XC_HF) {
        set_error("mess_batch_scf_create: exchange form %d is not built for batches", opts->xc);
        return MESS_E_UNSUPPORTED;
    }
    if (opts->diis_size < 0 || opts->diis_size > kBMaxDiis || !(opts->conv_tol >= 0.0)) {
        set_error("mess_batch_scf_create: diis_size must be 0..%d and conv_tol >= 0", kBMaxDiis);
        return MESS_E_ARG;
    }
    auto *st = new mess_batch_scf();
    st->basis = const_cast<mess_basis *>(basis);
    st->opts = *opts;
    st->use_graph = use_graph != 0;
    int rc = batch_create_impl(st, D0);
    if (rc != MESS_OK) {
        free_batch(st);
        return rc;
    }
    *out = st;
    return MESS_OK;
}

int mess_batch_scf_step(mess_batch_scf *st, mess_stream stream) {
    if (!st) {
        set_error("mess_batch_scf_step: NULL handle");
        return MESS_E_ARG;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    // kind of this step, decided on the host from the step count alone
    int kind = kStepFull64;
    if (st->opts.prec == MESS_FP32) {
        if (st->host_iter < kFarSteps) {
            kind = kStepFull32;
        } else if (st->host_iter == kFarSteps) {
            kind = kStepFull64Open;  // the previous energy was not anchored
            st->since_full = 0;
        } else if (st->since_full >= kDeltaRun) {
            kind = kStepFull64;
            st->since_full = 0;
        } else {
            kind = kStepDelta32;
            ++st->since_full;
        }
    }
    st->host_iter += 1;
    if (!st->use_graph) return enqueue_step(st, s, kind);
    if (!st->exec[kind]) {
        if (prof_on()) {
            set_error("mess_batch_scf_step: class profiling cannot be recorded inside a graph");
            return MESS_E_ARG;
        }
        MESS_HIP(hipStreamBeginCapture(st->cap, hipStreamCaptureModeThreadLocal));
        int rc = enqueue_step(st, st->cap, kind);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(st->cap, &g);
        if (rc != MESS_OK) {
            if (g) hipGraphDestroy(g);
            return rc;
        }
        MESS_HIP(e);
        st->graph[kind] = g;
        MESS_HIP(hipGraphInstantiate(&st->exec[kind], st->graph[kind], nullptr, nullptr, 0));
    }
    MESS_HIP(hipGraphLaunch(st->exec[kind], s));
    return MESS_OK;
}

int mess_batch_scf_status(const mess_batch_scf *st, double *energy, double *delta_e, double *resid,
                          int32_t *converged, int32_t *n_converged, mess_stream stream) {
    if (!st) {
        set_error("mess_batch_scf_status: NULL handle");
        return MESS_E_ARG;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<MolScalars> h(st->nmol);
    MESS_HIP(hipMemcpyAsync(h.data(), st->ms, sizeof(MolScalars) * st->nmol, hipMemcpyDeviceToHost, s));
    MESS_HIP(hipStreamSynchronize(s));
    int nc = 0, bad_sp2 = -1, bad_e = -1;
    for (int m = 0; m < st->nmol; ++m) {
        if (energy) energy[m] = h[m].energy;
        if (delta_e) delta_e[m] = h[m].de;
        if (resid) resid[m] = h[m].resid;
        if (converged) converged[m] = h[m].frozen;
        nc += h[m].frozen;
        if (h[m].sp2_fail && bad_sp2 < 0) bad_sp2 = m;
        if (!std::isfinite(h[m].energy) && bad_e < 0) bad_e = m;
    }
    if (n_converged) *n_converged = nc;
    if (bad_e >= 0) {
        set_error("mess_batch_scf_status: non-finite energy for molecule %d", bad_e);
        return MESS_E_NUMERIC;
    }
    if (bad_sp2 >= 0) {
        set_error("mess_batch_scf_status: density purification of molecule %d did not finish in %d rounds", bad_sp2,
                  kSp2Rounds);
        return MESS_E_NUMERIC;
    }
    return MESS_OK;
}

int mess_batch_scf_guard(const mess_batch_scf *st, int32_t *stage) {
    if (!st || !stage) {
        set_error("mess_batch_scf_guard: NULL argument");
        return MESS_E_ARG;
    }
    std::vector<MolScalars> h(st->nmol);
    MESS_HIP(hipMemcpy(h.data(), st->ms, sizeof(MolScalars) * st->nmol, hipMemcpyDeviceToHost));
    for (int m = 0; m < st->nmol; ++m) stage[m] = h[m].stage;
    return MESS_OK;
}

int mess_batch_scf_density(const mess_batch_scf *st, double *D, mess_stream stream) {
    if (!st || !D) {
        set_error("mess_batch_scf_density: NULL argument");
        return MESS_E_ARG;
    }
    MESS_HIP(hipMemcpyAsync(D, st->D, sizeof(double) * st->packed, hipMemcpyDeviceToDevice,
                            static_cast<hipStream_t>(stream)));
    return MESS_OK;
}

void mess_batch_scf_destroy(mess_batch_scf *st) { free_batch(st); }

}  // extern "C"
