// Self-consistent field iteration for the Roothaan equation F(C) C = S C eps
// (paper section 3, eq. 2), closed shell, on the device.
//
// Per step at density D_k:  J, K <- D_k;  F_k = H + J - K/2;
// E_k = 1/2 Tr[D_k (H + F_k)] + E_nuc;  commutator e_k = X^T (F D S - S D F) X;
// then (unless converged) optional Pulay DIIS on F, F' = X^T F X and the new
// density D_{k+1} = 2 X P X^T where P is the projector onto the n_occ lowest
// eigenvectors of F'.  X is the canonical orthogonaliser U s^{-1/2} over the
// eigenpairs of S with s > 1e-7 (eq. 5: C^T S C = 1 for C = X C').
//
// P is obtained without an eigensolver by trace-correcting second-order
// spectral projection: X_0 = (e_max - F') / (e_max - e_min) with Gershgorin
// bounds, then repeatedly X <- X^2 or X <- 2X - X^2, whichever moves the
// trace towards n_occ.  The fixed point is the same projector an aufbau
// occupation of the eigenvectors gives whenever the HOMO-LUMO gap is open.
#include <cmath>
#include <vector>

#include "class_ops.hpp"
#include "linalg.hpp"
#include "mess_internal.hpp"

namespace mess {

int jk_direct_half(mess_basis *B, const double *D, double *Gj, double *Gk, int prec, double tau, hipStream_t s);
int jk_stored(mess_basis *B, const double *D, double *Gj, double *Gk, int prec, double tau, hipStream_t s);
int jk_det(mess_basis *B, const double *D, double *Gj, double *Gk, int prec, double tau, hipStream_t s);
int zero_async(double *p, int64_t n, hipStream_t s);
int lda_x_async(mess_basis *B, const double *D, double *V, hipStream_t s, const double **ex_dev);
int pbe_xc_async(mess_basis *B, const double *D, double *V, hipStream_t s, const double **ex_dev);

constexpr int kMaxDiis = 16;

// Device scalars shared by the small kernels of one step.
struct ScfScalars {
    double energy, resid;
    double emin, emax;
    double trX, trX2;
    double idem;          // tr(X) - tr(X^2) of the last purification step
    double dmax;          // max |dD| of the last incremental build
    int sp2_iter, sp2_done, sp2_post;
    int flag;             // direct minimisation: Cholesky pivot not positive
    double diis_c[kMaxDiis + 1];
};

}  // namespace mess

struct mess_scf {
    mess_basis *basis = nullptr;
    mess_scf_opts opts{};
    int N = 0, M = 0;  // basis functions, orthonormal functions kept
    int iter = 0;
    double e_prev = 0.0;
    hipStream_t create_stream = nullptr;
    // device buffers
    double *S = nullptr, *H = nullptr, *X = nullptr, *D = nullptr, *F = nullptr, *Fx = nullptr;
    double *Gj = nullptr, *Gk = nullptr;
    double *W1 = nullptr, *W2 = nullptr, *W3 = nullptr;  // N x N work
    double *P = nullptr, *P2 = nullptr;                  // M x M purification
    double *Fh = nullptr, *Eh = nullptr;                 // DIIS history [kMaxDiis][N*N], [kMaxDiis][M*M]
    double *Bm = nullptr;                                // DIIS B matrix kMaxDiis^2
    mess::ScfScalars *sc = nullptr;
    double *partial = nullptr;                           // reduction partials
    double *Dprev = nullptr, *dD = nullptr, *Gja = nullptr, *Gka = nullptr;  // FP32 incremental builds
    double *Vx = nullptr;                                // LDA exchange / PBE exchange-correlation potential
    int *d_hs = nullptr;                                 // DIIS history slot list, kMaxDiis
    // direct minimisation (mess_dmin_step): trial matrix, QR factors, Adam
    // moments, gradient work (N x N each, built on the first call)
    double *Zt = nullptr, *Qf = nullptr, *Rf = nullptr, *Am = nullptr, *Av = nullptr, *Gz = nullptr;
    int dmin_t = 0;
    double last_de = 1e300;  // |E_k - E_{k-1}| of the previous step
    double last_dmax = 0.0;  // max |dD| and screening threshold of the last incremental build
    double last_tau = 0.0;
    bool acc_valid = false;   // FP32 mode: Gja/Gka hold an FP64 build plus dD builds
    bool near = false;        // FP32 mode: the energy change has been below kNearDe
    bool prev_anchored = false;  // FP32 mode: the previous energy came from anchored J/K
    int since_full = 0;       // dD builds since the last complete build
    int last_build_prec = 0;  // last Fock build: MESS_FP64/MESS_FP32 complete, -prec-1 for a dD build
    std::vector<int> hist;  // history slots, oldest first
    int next_slot = 0;
    int sp2_iters_last = 0;
    // divergence guard: stage 0 DIIS, 1 DIIS afresh, 2 damped DIIS, 3
    // restarted from the core guess (damped); rises of the energy counted
    // since the stage began; whether e_prev holds an energy to compare with
    int stage = 0, rises = 0;
    bool have_prev = false;
};

namespace mess {

constexpr int kRedBlocks = 256;
// Mixed precision: energy change below which the Fock builds switch from
// complete FP32 builds to an FP64 build plus FP32 builds of the density
// change (Hartree).
constexpr double kNearDe = 1e-1;
// Divergence guard: from iteration kGuardFrom on, an energy rise above kRiseTol (Hartree) counts against
// the current stage, kRisesPerStage of them move to the next stage; from
// stage 2 the next density is mixed with the current one with weight kDamp.
constexpr double kRiseTol = 1e-6;
constexpr int kRisesPerStage = 2;
constexpr int kGuardFrom = 12;  // rises count from this iteration on (DIIS settles first)
constexpr double kDamp = 0.5;

// Hartree-Fock (Vx == NULL): F = H + J - K/2 with J = Gj + Gj^T,
// K = Gk + Gk^T, and per-block partial sums of D .* (H + F);
// LDA exchange or PBE exchange-correlation: F = H + J + Vx and partial sums of D .* (2H + J), so that
// half the total is Tr[D H] + 1/2 Tr[D J] in both cases (deterministic
// two-stage reduction).
__global__ void __launch_bounds__(256) k_fock(int N, const double *__restrict__ H, const double *__restrict__ Gj,
                                              const double *__restrict__ Gk, const double *__restrict__ Vx,
                                              const double *__restrict__ D, double *__restrict__ F,
                                              double *__restrict__ partial) {
    __shared__ double red[256];
    double acc = 0.0;
    const int64_t NN = (int64_t)N * N;
    for (int64_t idx = blockIdx.x * 256 + threadIdx.x; idx < NN; idx += (int64_t)gridDim.x * 256) {
        const int i = (int)(idx / N), j = (int)(idx % N);
        const int64_t t = (int64_t)j * N + i;
        const double J = Gj[idx] + Gj[t];
        if (Vx) {
            F[idx] = H[idx] + J + Vx[idx];
            acc += D[idx] * (2.0 * H[idx] + J);
        } else {
            const double f = H[idx] + J - 0.5 * (Gk[idx] + Gk[t]);
            F[idx] = f;
            acc += D[idx] * (H[idx] + f);
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) k_finish_energy(int nblk, const double *__restrict__ partial, double enuc,
                                                       const double *__restrict__ ex, ScfScalars *__restrict__ sc) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nblk; i += 256) acc += partial[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) sc->energy = 0.5 * red[0] + enuc + (ex ? ex[0] : 0.0);
}

// C = M - M^T
__global__ void k_antisym(int N, const double *__restrict__ Mx, double *__restrict__ C) {
    const int64_t NN = (int64_t)N * N;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < NN; idx += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(idx / N), j = (int)(idx % N);
        C[idx] = Mx[idx] - Mx[(int64_t)j * N + i];
    }
}

// max |x| over n values -> sc->resid (single block, 1024 threads)
__global__ void __launch_bounds__(1024) k_maxabs(int64_t n, const double *__restrict__ x, ScfScalars *__restrict__ sc) {
    __shared__ double red[1024];
    double m = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) m = fmax(m, fabs(x[i]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int st = 512; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0) sc->resid = red[0];
}

// max |x| over n values -> *out (single block, 1024 threads)
__global__ void __launch_bounds__(1024) k_maxabs_to(int64_t n, const double *__restrict__ x, double *__restrict__ out) {
    __shared__ double red[1024];
    double m = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) m = fmax(m, fabs(x[i]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int st = 512; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// B[slot][k] = B[k][slot] = <E_slot, E_k> for the listed history slots.
__global__ void __launch_bounds__(256) k_diis_dots(int64_t n, int slot, const int *__restrict__ slots, int nslots,
                                                   const double *__restrict__ Eh, double *__restrict__ Bm) {
    __shared__ double red[256];
    const int k = slots[blockIdx.x];
    const double *a = Eh + (int64_t)slot * n, *b = Eh + (int64_t)k * n;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) acc += a[i] * b[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        Bm[slot * kMaxDiis + k] = red[0];
        Bm[k * kMaxDiis + slot] = red[0];
    }
}

// Solve [[B, -1], [-1^T, 0]] [c; lambda] = [0; -1] by Gaussian elimination
// with partial pivoting (one thread; m <= kMaxDiis).
__global__ void k_diis_solve(int m, const int *__restrict__ slots, const double *__restrict__ Bm,
                             ScfScalars *__restrict__ sc) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double A[kMaxDiis + 1][kMaxDiis + 2];
    const int n = m + 1;
    for (int i = 0; i < m; ++i) {
        for (int j = 0; j < m; ++j) A[i][j] = Bm[slots[i] * kMaxDiis + slots[j]];
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
    double x[kMaxDiis + 1];
    for (int r = n - 1; r >= 0; --r) {
        double s = A[r][n];
        for (int c = r + 1; c < n; ++c) s -= A[r][c] * x[c];
        x[r] = A[r][r] != 0.0 ? s / A[r][r] : 0.0;
    }
    for (int i = 0; i < m; ++i) sc->diis_c[i] = x[i];
}

// Fx = sum_i c_i Fh[slot_i]
__global__ void k_diis_combine(int64_t n, int m, const int *__restrict__ slots, const double *__restrict__ Fh,
                               const ScfScalars *__restrict__ sc, double *__restrict__ Fx) {
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n; idx += (int64_t)gridDim.x * blockDim.x) {
        double v = 0.0;
        for (int i = 0; i < m; ++i) v += sc->diis_c[i] * Fh[(int64_t)slots[i] * n + idx];
        Fx[idx] = v;
    }
}

// Gershgorin bounds of a symmetric M x M matrix (one block).
__global__ void __launch_bounds__(1024) k_gershgorin(int M, const double *__restrict__ A, ScfScalars *__restrict__ sc) {
    __shared__ double lo[1024], hi[1024];
    double l = 1e300, h = -1e300;
    for (int i = threadIdx.x; i < M; i += 1024) {
        double r = 0.0;
        for (int j = 0; j < M; ++j)
            if (j != i) r += fabs(A[(int64_t)i * M + j]);
        const double d = A[(int64_t)i * M + i];
        l = fmin(l, d - r);
        h = fmax(h, d + r);
    }
    lo[threadIdx.x] = l;
    hi[threadIdx.x] = h;
    __syncthreads();
    for (int st = 512; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            lo[threadIdx.x] = fmin(lo[threadIdx.x], lo[threadIdx.x + st]);
            hi[threadIdx.x] = fmax(hi[threadIdx.x], hi[threadIdx.x + st]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        sc->emin = lo[0];
        sc->emax = hi[0] > lo[0] ? hi[0] : lo[0] + 1.0;
        sc->sp2_iter = 0;
        sc->sp2_done = 0;
        sc->sp2_post = 0;
    }
}

// X0 = (e_max I - F') / (e_max - e_min)
__global__ void k_sp2_init(int M, const double *__restrict__ Fp, const ScfScalars *__restrict__ sc,
                           double *__restrict__ X) {
    const double emax = sc->emax, inv = 1.0 / (sc->emax - sc->emin);
    const int64_t MM = (int64_t)M * M;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < MM; idx += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(idx / M), j = (int)(idx % M);
        X[idx] = ((i == j ? emax : 0.0) - Fp[idx]) * inv;
    }
}

// traces of X and X2 (one block)
__global__ void __launch_bounds__(1024) k_sp2_traces(int M, const double *__restrict__ X, const double *__restrict__ X2,
                                                     ScfScalars *__restrict__ sc) {
    __shared__ double a[1024], b[1024];
    if (sc->sp2_done) return;
    double s1 = 0.0, s2 = 0.0;
    for (int i = threadIdx.x; i < M; i += 1024) {
        s1 += X[(int64_t)i * M + i];
        s2 += X2[(int64_t)i * M + i];
    }
    a[threadIdx.x] = s1;
    b[threadIdx.x] = s2;
    __syncthreads();
    for (int st = 512; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            a[threadIdx.x] += a[threadIdx.x + st];
            b[threadIdx.x] += b[threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        sc->trX = a[0];
        sc->trX2 = b[0];
        sc->idem = a[0] - b[0];
    }
}

// X <- X^2 or 2X - X^2 (trace towards n_occ); convergence bookkeeping.
__global__ void k_sp2_update(int M, double nocc, double *__restrict__ X, const double *__restrict__ X2,
                             ScfScalars *__restrict__ sc) {
    if (sc->sp2_done) return;
    const double t1 = sc->trX, t2 = sc->trX2;
    const bool square = fabs(t2 - nocc) < fabs(2.0 * t1 - t2 - nocc);
    const int64_t MM = (int64_t)M * M;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < MM; idx += (int64_t)gridDim.x * blockDim.x)
        X[idx] = square ? X2[idx] : 2.0 * X[idx] - X2[idx];
}

__global__ void k_sp2_bookkeep(ScfScalars *__restrict__ sc) {
    if (threadIdx.x != 0 || sc->sp2_done) return;
    sc->sp2_iter += 1;
    // once idempotent to 1e-10, two more quadratic steps reach rounding level
    if (sc->sp2_post > 0 || fabs(sc->idem) < 1e-10) sc->sp2_post += 1;
    if (sc->sp2_post >= 3) sc->sp2_done = 1;
}

__global__ void k_scale_identity_minus(int M, double a, double b, const double *__restrict__ Z, double *__restrict__ out) {
    // out = a I + b Z
    const int64_t MM = (int64_t)M * M;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < MM; idx += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(idx / M), j = (int)(idx % M);
        out[idx] = (i == j ? a : 0.0) + b * Z[idx];
    }
}

// X[:, k] = U[:, drop + k] / sqrt(w[drop + k]), N x M
__global__ void k_canonical_x(int N, int M, int drop, const double *__restrict__ U, const double *__restrict__ w,
                              double *__restrict__ X) {
    const int64_t n = (int64_t)N * M;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n; idx += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(idx / M), k = (int)(idx % M);
        X[idx] = U[(int64_t)i * N + drop + k] / sqrt(w[drop + k]);
    }
}

// r = max |A - I| (single block)
__global__ void __launch_bounds__(1024) k_maxabs_minus_identity(int N, const double *__restrict__ A,
                                                                ScfScalars *__restrict__ sc) {
    __shared__ double red[1024];
    double m = 0.0;
    const int64_t NN = (int64_t)N * N;
    for (int64_t i = threadIdx.x; i < NN; i += 1024) m = fmax(m, fabs(A[i] - ((i / N == i % N) ? 1.0 : 0.0)));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int st = 512; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0) sc->resid = red[0];
}

// max row sum of |A| (infinity norm, single block) -> sc->trX
__global__ void __launch_bounds__(1024) k_norm_inf(int N, const double *__restrict__ A, ScfScalars *__restrict__ sc) {
    __shared__ double red[1024];
    double m = 0.0;
    for (int i = threadIdx.x; i < N; i += 1024) {
        double r = 0.0;
        for (int j = 0; j < N; ++j) r += fabs(A[(int64_t)i * N + j]);
        m = fmax(m, r);
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int st = 512; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0) sc->trX = red[0];
}

__global__ void k_identity_scaled(int N, double a, const double *__restrict__ src, double *__restrict__ out) {
    // out = a * src (src != NULL) or the identity (src == NULL)
    const int64_t NN = (int64_t)N * N;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < NN; idx += (int64_t)gridDim.x * blockDim.x)
        out[idx] = src ? a * src[idx] : ((idx / N == idx % N) ? 1.0 : 0.0);
}

static unsigned grid1(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g > 2048) g = 2048;
    return (unsigned)(g < 1 ? 1 : g);
}

// Projector P (M x M) onto the n_occ lowest eigenvectors of Fp; P and P2
// are work buffers (result in P).  Returns the number of iterations.
static int purify(mess_scf *st, const double *Fp, hipStream_t s, int *iters) {
    const int M = st->M;
    const double nocc = st->basis->nocc;
    hipLaunchKernelGGL(k_gershgorin, dim3(1), dim3(1024), 0, s, M, Fp, st->sc);
    hipLaunchKernelGGL(k_sp2_init, dim3(grid1((int64_t)M * M)), dim3(256), 0, s, M, Fp, st->sc, st->P);
    MESS_LAUNCH_CHECK();
    const int chunk = 8, maxit = 200;
    int done = 0, it = 0;
    while (!done && it < maxit) {
        for (int k = 0; k < chunk; ++k) {
            MESS_TRY(gemm(s, false, false, M, M, M, 1.0, st->P, M, st->P, M, 0.0, st->P2, M));
            hipLaunchKernelGGL(k_sp2_traces, dim3(1), dim3(1024), 0, s, M, st->P, st->P2, st->sc);
            hipLaunchKernelGGL(k_sp2_update, dim3(grid1((int64_t)M * M)), dim3(256), 0, s, M, nocc, st->P, st->P2,
                               st->sc);
            hipLaunchKernelGGL(k_sp2_bookkeep, dim3(1), dim3(64), 0, s, st->sc);
        }
        MESS_LAUNCH_CHECK();
        it += chunk;
        MESS_HIP(hipMemcpyAsync(&done, &st->sc->sp2_done, sizeof(int), hipMemcpyDeviceToHost, s));
        MESS_HIP(hipStreamSynchronize(s));
    }
    int n = 0;
    MESS_HIP(hipMemcpyAsync(&n, &st->sc->sp2_iter, sizeof(int), hipMemcpyDeviceToHost, s));
    MESS_HIP(hipStreamSynchronize(s));
    *iters = n;
    return MESS_OK;
}

// D = 2 X P X^T from the projector in the orthonormal basis.
static int density_from_projector(mess_scf *st, hipStream_t s, double *Dout) {
    const int N = st->N, M = st->M;
    MESS_TRY(gemm(s, false, false, N, M, M, 1.0, st->X, M, st->P, M, 0.0, st->W1, M));      // W1 = X P  (N x M)
    MESS_TRY(gemm(s, false, true, N, N, M, 2.0, st->W1, M, st->X, M, 0.0, Dout, N));       // D = 2 W1 X^T
    return MESS_OK;
}

// Fp = X^T F X (M x M) into P2's partner buffer W2.
static int to_orthonormal(mess_scf *st, const double *F, double *Fp, hipStream_t s) {
    const int N = st->N, M = st->M;
    MESS_TRY(gemm(s, true, false, M, N, N, 1.0, st->X, M, F, N, 0.0, st->W3, N));   // W3 = X^T F (M x N)
    MESS_TRY(gemm(s, false, false, M, M, N, 1.0, st->W3, N, st->X, M, 0.0, Fp, M));  // Fp = W3 X
    return MESS_OK;
}

// Core-Hamiltonian guess: D from the aufbau projector of X^T H X.
static int core_density(mess_scf *st, hipStream_t s) {
    MESS_TRY(to_orthonormal(st, st->H, st->W2, s));
    int it = 0;
    MESS_TRY(purify(st, st->W2, s, &it));
    return density_from_projector(st, s, st->D);
}

// Loewdin orthogonaliser X = S^{-1/2} by the coupled Newton-Schulz
// iteration on A = S / c (c >= lambda_max(S) by Gershgorin, so the spectrum
// of A lies in (0, 1]):  T = (3 I - Z Y)/2,  Y <- Y T,  Z <- T Z, from
// Y = A, Z = I; Z -> A^{-1/2}.  *ok is false if it did not converge or if
// lambda_min(S) >= 1 / ||S^{-1}||_inf cannot be shown to exceed 1e-6 (then
// the caller uses the eigensolver and canonical dropping instead).
static int lowdin_newton_schulz(mess_scf *st, hipStream_t s, bool *ok) {
    const int N = st->N;
    const int64_t nn = (int64_t)N * N;
    *ok = false;
    hipLaunchKernelGGL(k_gershgorin, dim3(1), dim3(1024), 0, s, N, st->S, st->sc);
    ScfScalars h;
    MESS_HIP(hipMemcpyAsync(&h, st->sc, sizeof(ScfScalars), hipMemcpyDeviceToHost, s));
    MESS_HIP(hipStreamSynchronize(s));
    const double c = h.emax;
    if (!(c > 0.0) || !std::isfinite(c)) return MESS_OK;
    double *Y = st->Gj, *Z = st->Gk, *T = st->F, *tmp = st->Fx;
    hipLaunchKernelGGL(k_identity_scaled, dim3(grid1(nn)), dim3(256), 0, s, N, 1.0 / c, st->S, Y);
    hipLaunchKernelGGL(k_identity_scaled, dim3(grid1(nn)), dim3(256), 0, s, N, 0.0, nullptr, Z);
    MESS_LAUNCH_CHECK();
    bool conv = false;
    for (int it = 0; it < 80 && !conv; ++it) {
        MESS_TRY(gemm(s, false, false, N, N, N, 1.0, Z, N, Y, N, 0.0, tmp, N));  // tmp = Z Y
        if (it % 4 == 3) {
            hipLaunchKernelGGL(k_maxabs_minus_identity, dim3(1), dim3(1024), 0, s, N, tmp, st->sc);
            MESS_HIP(hipMemcpyAsync(&h, st->sc, sizeof(ScfScalars), hipMemcpyDeviceToHost, s));
            MESS_HIP(hipStreamSynchronize(s));
            if (!std::isfinite(h.resid)) return MESS_OK;
            if (h.resid < 1e-14) conv = true;
        }
        hipLaunchKernelGGL(k_scale_identity_minus, dim3(grid1(nn)), dim3(256), 0, s, N, 1.5, -0.5, tmp, T);
        MESS_TRY(gemm(s, false, false, N, N, N, 1.0, Y, N, T, N, 0.0, tmp, N));  // Y T
        std::swap(Y, tmp);
        MESS_TRY(gemm(s, false, false, N, N, N, 1.0, T, N, Z, N, 0.0, tmp, N));  // T Z
        std::swap(Z, tmp);
    }
    if (!conv) return MESS_OK;
    // X = Z / sqrt(c); bound lambda_min(S) >= 1/||X X||_inf
    hipLaunchKernelGGL(k_identity_scaled, dim3(grid1(nn)), dim3(256), 0, s, N, 1.0 / std::sqrt(c), Z, st->X);
    MESS_LAUNCH_CHECK();
    MESS_TRY(gemm(s, false, false, N, N, N, 1.0, st->X, N, st->X, N, 0.0, tmp, N));
    hipLaunchKernelGGL(k_norm_inf, dim3(1), dim3(1024), 0, s, N, tmp, st->sc);
    MESS_HIP(hipMemcpyAsync(&h, st->sc, sizeof(ScfScalars), hipMemcpyDeviceToHost, s));
    MESS_HIP(hipStreamSynchronize(s));
    if (std::isfinite(h.trX) && h.trX > 0.0 && 1.0 / h.trX > 1e-6) {
        st->M = N;
        *ok = true;
    }
    return MESS_OK;
}

static void free_scf(mess_scf *st) {
    if (!st) return;
    for (double *p : {st->S, st->H, st->X, st->D, st->F, st->Fx, st->Gj, st->Gk, st->W1, st->W2, st->W3, st->P,
                      st->P2, st->Fh, st->Eh, st->Bm, st->partial, st->Dprev, st->dD, st->Gja, st->Gka, st->Vx})
        hipFree(p);
    hipFree(st->sc);
    hipFree(st->d_hs);
    for (double *p : {st->Zt, st->Qf, st->Rf, st->Am, st->Av, st->Gz}) hipFree(p);
    delete st;
}

// Canonical orthogonaliser X = U s^{-1/2} over the eigenpairs of S with
// s > 1e-7, from the one-workgroup Jacobi eigensolver.
static int canonical_orthogonaliser(mess_scf *st, hipStream_t s) {
    mess_basis *B = st->basis;
    const int N = st->N;
    const size_t nn = (size_t)N * N;
    MESS_HIP(hipMemcpyAsync(st->W1, st->S, sizeof(double) * nn, hipMemcpyDeviceToDevice, s));
    std::vector<double> wh(N);
    double *wdev = nullptr;
    MESS_HIP(hipMalloc(&wdev, sizeof(double) * N));
    double *work = nullptr;
    MESS_HIP(hipMalloc(&work, sizeof(double) * (nn + N)));
    int rc = jacobi_eigh(s, N, st->W1, wdev, st->W2, work);
    if (rc == MESS_OK && hipMemcpyAsync(wh.data(), wdev, sizeof(double) * N, hipMemcpyDeviceToHost, s) != hipSuccess)
        rc = MESS_E_DEVICE;
    if (rc == MESS_OK && hipStreamSynchronize(s) != hipSuccess) rc = MESS_E_DEVICE;
    int drop = 0;
    if (rc == MESS_OK) {
        for (int i = 0; i < N; ++i)
            if (!std::isfinite(wh[i])) {
                set_error("mess_scf_create: non-finite overlap eigenvalue");
                rc = MESS_E_NUMERIC;
                break;
            }
        while (rc == MESS_OK && drop < N && wh[drop] <= 1e-7) ++drop;
    }
    if (rc == MESS_OK) {
        st->M = N - drop;
        if (st->M < B->nocc || st->M <= 0) {
            set_error("mess_scf_create: only %d linearly independent functions for %d occupied orbitals", st->M,
                      B->nocc);
            rc = MESS_E_NUMERIC;
        }
    }
    if (rc == MESS_OK) {
        hipLaunchKernelGGL(k_canonical_x, dim3(grid1((int64_t)N * st->M)), dim3(256), 0, s, N, st->M, drop, st->W2,
                           wdev, st->X);
        if (hipGetLastError() != hipSuccess) rc = MESS_E_DEVICE;
    }
    hipStreamSynchronize(s);
    hipFree(wdev);
    hipFree(work);
    if (rc != MESS_OK) {
        if (rc == MESS_E_DEVICE) set_error("mess_scf_create: device error in the overlap eigensolve");
        return rc;
    }
    return MESS_OK;
}

static int scf_create_impl(mess_scf *st, const double *D0) {
    mess_basis *B = st->basis;
    const int N = B->nbf;
    st->N = N;
    hipStream_t s = nullptr;
    const size_t nn = (size_t)N * N;
    for (double **p : {&st->S, &st->H, &st->X, &st->D, &st->F, &st->Fx, &st->Gj, &st->Gk, &st->W1, &st->W2, &st->W3,
                       &st->P, &st->P2})
        MESS_HIP(hipMalloc(p, sizeof(double) * std::max<size_t>(nn, 16)));
    const int nd = std::max(1, std::min(st->opts.diis_size, kMaxDiis));
    MESS_HIP(hipMalloc(&st->Fh, sizeof(double) * nn * nd));
    MESS_HIP(hipMalloc(&st->Eh, sizeof(double) * nn * nd));
    MESS_HIP(hipMalloc(&st->Bm, sizeof(double) * kMaxDiis * kMaxDiis));
    MESS_HIP(hipMalloc(&st->d_hs, sizeof(int) * kMaxDiis));
    if (st->opts.prec == MESS_FP32)
        for (double **p : {&st->Dprev, &st->dD, &st->Gja, &st->Gka})
            MESS_HIP(hipMalloc(p, sizeof(double) * std::max<size_t>(nn, 16)));
    if (st->opts.xc != MESS_XC_HF) MESS_HIP(hipMalloc(&st->Vx, sizeof(double) * std::max<size_t>(nn, 16)));
    MESS_HIP(hipMalloc(&st->sc, sizeof(ScfScalars)));
    MESS_HIP(hipMalloc(&st->partial, sizeof(double) * kRedBlocks));
    MESS_HIP(hipMemset(st->sc, 0, sizeof(ScfScalars)));
    // one-electron: S in S, T in W1, V in W2 -> H
    MESS_TRY(mess_one_electron(B, st->S, st->W1, st->W2, s));
    MESS_TRY(axpby(s, (int64_t)nn, 1.0, st->W1, 1.0, st->W2, st->H));
    // Loewdin orthogonaliser by Newton-Schulz; eigensolver + canonical
    // dropping only when S may be near-singular
    bool lowdin = false;
    MESS_TRY(lowdin_newton_schulz(st, s, &lowdin));
    if (!lowdin) MESS_TRY(canonical_orthogonaliser(st, s));
    const int M = st->M;
    // two Newton steps X <- X (3 I - X^T S X) / 2 restore X^T S X = I to rounding
    for (int k = 0; k < 2; ++k) {
        MESS_TRY(gemm(s, false, false, N, M, N, 1.0, st->S, N, st->X, M, 0.0, st->W1, M));   // W1 = S X
        MESS_TRY(gemm(s, true, false, M, M, N, 1.0, st->X, M, st->W1, M, 0.0, st->P, M));    // P = X^T S X
        hipLaunchKernelGGL(k_scale_identity_minus, dim3(grid1((int64_t)M * M)), dim3(256), 0, s, M, 1.5, -0.5, st->P,
                           st->P2);
        MESS_TRY(gemm(s, false, false, N, M, M, 1.0, st->X, M, st->P2, M, 0.0, st->W1, M));  // W1 = X (1.5 - 0.5 Z)
        MESS_HIP(hipMemcpyAsync(st->X, st->W1, sizeof(double) * N * M, hipMemcpyDeviceToDevice, s));
    }
    // initial density
    if (D0) {
        MESS_HIP(hipMemcpyAsync(st->D, D0, sizeof(double) * nn, hipMemcpyDeviceToDevice, s));
    } else {
        MESS_TRY(core_density(st, s));
    }
    MESS_HIP(hipStreamSynchronize(s));
    return MESS_OK;
}

// Last stage of the divergence guard: the density restarts from the core
// guess, the DIIS history is dropped, the next energy is compared with
// nothing and (mixed precision) the next build is a complete one.
static int scf_restart(mess_scf *st, hipStream_t s) {
    st->stage = 3;
    st->rises = 0;
    st->hist.clear();
    st->next_slot = 0;
    st->have_prev = false;
    st->acc_valid = false;
    MESS_TRY(core_density(st, s));
    MESS_HIP(hipStreamSynchronize(s));
    return MESS_OK;
}

static bool scf_deterministic(const mess_scf *st) {
    return st->opts.deterministic != 0 || st->opts.jk_mode == MESS_JK_DETERMINISTIC;
}

// J/K half matrices of one Fock build in the state's mode: deterministic
// (stored blocks, exact accumulation, always at the options' threshold),
// direct or stored.
static int scf_jk(mess_scf *st, const double *D, double *Gj, double *Gk, int prec, double tau, hipStream_t s) {
    mess_basis *B = st->basis;
    if (scf_deterministic(st)) return jk_det(B, D, Gj, Gk, prec, st->opts.schwarz_tol, s);
    if (st->opts.jk_mode == MESS_JK_DIRECT) return jk_direct_half(B, D, Gj, Gk, prec, tau, s);
    return jk_stored(B, D, Gj, Gk, prec, tau, s);
}

static int scf_step_impl(mess_scf *st, double *energy, double *delta_e, double *resid, int32_t *converged,
                         hipStream_t s) {
    mess_basis *B = st->basis;
    const int N = st->N, M = st->M;
    const int64_t nn = (int64_t)N * N, mm = (int64_t)M * M;
    // J, K half matrices
    if (st->opts.prec == MESS_FP32) {
        // Mixed precision.  Until the energy change first drops below
        // kNearDe, every Fock build is a complete FP32 build (its rounding is
        // far below the change of the density, and nothing of it is kept).
        // From then on (for good) the first build is a complete FP64 build;
        // after it, builds of dD = D_k - D_{k-1} in FP32 are added to the
        // FP64 running half-matrices (their rounding scales with the small
        // change), with a complete FP64 rebuild after every 8 of them.
        // Convergence is only declared on FP64-anchored builds.
        if (st->last_de < kNearDe) st->near = true;
        const bool near = st->near;
        if (!near || !st->acc_valid || st->since_full >= 8) {
            const int fprec = near ? MESS_FP64 : MESS_FP32;
            MESS_TRY(scf_jk(st, st->D, st->Gja, st->Gka, fprec, st->opts.schwarz_tol, s));
            st->acc_valid = near;
            st->since_full = 0;
            st->last_build_prec = fprec;
        } else {
            const int dprec = MESS_FP32;
            st->last_build_prec = -dprec - 1;
            ++st->since_full;
            MESS_TRY(axpby(s, nn, 1.0, st->D, -1.0, st->Dprev, st->dD));
            // Direct builds screen the change by its size as well: a quartet
            // with Q_ab Q_cd max|dD| < tol moves no element of J or K by more
            // than a few tol, so the work list of tol / max|dD| (rounded down
            // to a power of ten, so that lists are reused) leaves out only
            // such quartets.  Stored blocks keep the list they were built for.
            double tau = st->opts.schwarz_tol;
            bool none = false;
            if (st->opts.jk_mode == MESS_JK_DIRECT && !scf_deterministic(st) && tau > 0.0) {
                hipLaunchKernelGGL(k_maxabs_to, dim3(1), dim3(1024), 0, s, nn, st->dD, &st->sc->dmax);
                MESS_LAUNCH_CHECK();
                double dmax = 0.0;
                MESS_HIP(hipMemcpyAsync(&dmax, &st->sc->dmax, sizeof(double), hipMemcpyDeviceToHost, s));
                MESS_HIP(hipStreamSynchronize(s));
                if (!std::isfinite(dmax)) {
                    set_error("mess_scf_step: non-finite density change");
                    return MESS_E_NUMERIC;
                }
                if (dmax == 0.0) none = true;
                else tau = std::pow(10.0, std::floor(std::log10(tau / dmax)));
                st->last_dmax = dmax;
                st->last_tau = none ? 0.0 : tau;
            }
            if (!none) {
                MESS_TRY(scf_jk(st, st->dD, st->Gj, st->Gk, dprec, tau, s));
                MESS_TRY(axpby(s, nn, 1.0, st->Gja, 1.0, st->Gj, st->Gja));
                MESS_TRY(axpby(s, nn, 1.0, st->Gka, 1.0, st->Gk, st->Gka));
            }
        }
        MESS_HIP(hipMemcpyAsync(st->Dprev, st->D, sizeof(double) * nn, hipMemcpyDeviceToDevice, s));
        MESS_HIP(hipMemcpyAsync(st->Gj, st->Gja, sizeof(double) * nn, hipMemcpyDeviceToDevice, s));
        MESS_HIP(hipMemcpyAsync(st->Gk, st->Gka, sizeof(double) * nn, hipMemcpyDeviceToDevice, s));
    } else {
        // LDA exchange needs no K
        double *Gk = st->Vx ? nullptr : st->Gk;
        MESS_TRY(scf_jk(st, st->D, st->Gj, Gk, st->opts.prec, st->opts.schwarz_tol, s));
    }
    const double *ex = nullptr;
    if (st->opts.xc == MESS_XC_LDA_X) MESS_TRY(lda_x_async(B, st->D, st->Vx, s, &ex));
    if (st->opts.xc == MESS_XC_PBE) MESS_TRY(pbe_xc_async(B, st->D, st->Vx, s, &ex));
    hipLaunchKernelGGL(k_fock, dim3(kRedBlocks), dim3(256), 0, s, N, st->H, st->Gj, st->Gk, st->Vx, st->D, st->F,
                       st->partial);
    hipLaunchKernelGGL(k_finish_energy, dim3(1), dim3(256), 0, s, kRedBlocks, st->partial, B->enuc, ex, st->sc);
    MESS_LAUNCH_CHECK();
    // commutator e = X^T (F D S - S D F) X, stored at the next DIIS slot
    const int nd = std::min(st->opts.diis_size, kMaxDiis);
    const int slot = nd > 0 ? st->next_slot : 0;
    double *e = nd > 0 ? st->Eh + (int64_t)slot * mm : st->P2;
    MESS_TRY(gemm(s, false, false, N, N, N, 1.0, st->F, N, st->D, N, 0.0, st->W1, N));    // W1 = F D
    MESS_TRY(gemm(s, false, false, N, N, N, 1.0, st->W1, N, st->S, N, 0.0, st->W2, N));   // W2 = F D S
    hipLaunchKernelGGL(k_antisym, dim3(grid1(nn)), dim3(256), 0, s, N, st->W2, st->W1);  // W1 = W2 - W2^T
    MESS_TRY(gemm(s, true, false, M, N, N, 1.0, st->X, M, st->W1, N, 0.0, st->W3, N));    // W3 = X^T W1
    MESS_TRY(gemm(s, false, false, M, M, N, 1.0, st->W3, N, st->X, M, 0.0, e, M));       // e = W3 X
    hipLaunchKernelGGL(k_maxabs, dim3(1), dim3(1024), 0, s, mm, e, st->sc);
    MESS_LAUNCH_CHECK();
    ScfScalars h;
    MESS_HIP(hipMemcpyAsync(&h, st->sc, sizeof(ScfScalars), hipMemcpyDeviceToHost, s));
    MESS_HIP(hipStreamSynchronize(s));
    const bool guard = st->opts.no_guard == 0;
    if (!std::isfinite(h.energy)) {
        if (!guard || st->stage >= 3) {
            set_error("mess_scf_step: non-finite energy");
            return MESS_E_NUMERIC;
        }
        // divergence guard: straight to the restart from the core guess
        if (energy) *energy = h.energy;
        if (delta_e) *delta_e = 0.0;
        if (resid) *resid = h.resid;
        if (converged) *converged = 0;
        st->iter += 1;
        st->last_de = 1e300;
        return scf_restart(st, s);
    }
    const bool have_prev = st->have_prev;
    const double de = have_prev ? h.energy - st->e_prev : 0.0;
    // mixed precision: only an energy on FP64-anchored J/K, following
    // another such energy, may end the iteration
    const bool anchored = st->opts.prec != MESS_FP32 || (st->acc_valid && st->prev_anchored);
    const bool conv = have_prev && std::fabs(de) < st->opts.conv_tol && anchored;
    st->prev_anchored = st->opts.prec != MESS_FP32 || st->acc_valid;
    if (energy) *energy = h.energy;
    if (delta_e) *delta_e = de;
    if (resid) *resid = h.resid;
    if (converged) *converged = conv ? 1 : 0;
    st->e_prev = h.energy;
    st->have_prev = true;
    st->last_de = have_prev ? std::fabs(de) : 1e300;
    st->iter += 1;
    if (conv) return MESS_OK;  // D stays the density that gave E_k
    // divergence guard: the second rise of the energy in a stage moves to
    // the next one (DIIS history dropped); the last stage restarts
    if (guard && have_prev && st->iter - 1 >= kGuardFrom && de > kRiseTol && ++st->rises >= kRisesPerStage &&
        st->stage < 3) {
        st->stage += 1;
        st->rises = 0;
        st->hist.clear();
        st->next_slot = 0;
        if (st->stage == 3) return scf_restart(st, s);
    }
    // DIIS
    const double *Fuse = st->F;
    if (nd > 0) {
        MESS_HIP(hipMemcpyAsync(st->Fh + (int64_t)slot * nn, st->F, sizeof(double) * nn, hipMemcpyDeviceToDevice, s));
        st->hist.push_back(slot);
        if ((int)st->hist.size() > nd) st->hist.erase(st->hist.begin());
        st->next_slot = (slot + 1) % nd;
        int hs[kMaxDiis];
        for (size_t i = 0; i < st->hist.size(); ++i) hs[i] = st->hist[i];
        int *d_hs = st->d_hs;
        int rc = MESS_OK;
        if (hipMemcpyAsync(d_hs, hs, sizeof(int) * st->hist.size(), hipMemcpyHostToDevice, s) != hipSuccess)
            rc = MESS_E_DEVICE;
        if (rc == MESS_OK) {
            hipLaunchKernelGGL(k_diis_dots, dim3((unsigned)st->hist.size()), dim3(256), 0, s, mm, slot, d_hs,
                               (int)st->hist.size(), st->Eh, st->Bm);
            if (st->hist.size() >= 2) {
                hipLaunchKernelGGL(k_diis_solve, dim3(1), dim3(64), 0, s, (int)st->hist.size(), d_hs, st->Bm, st->sc);
                hipLaunchKernelGGL(k_diis_combine, dim3(grid1(nn)), dim3(256), 0, s, nn, (int)st->hist.size(), d_hs,
                                   st->Fh, st->sc, st->Fx);
                Fuse = st->Fx;
            }
            if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) rc = MESS_E_DEVICE;
        }
        if (rc != MESS_OK) {
            set_error("mess_scf_step: DIIS kernels failed");
            return rc;
        }
    }
    MESS_TRY(to_orthonormal(st, Fuse, st->W2, s));
    int it = 0;
    MESS_TRY(purify(st, st->W2, s, &it));
    st->sp2_iters_last = it;
    if (st->stage >= 2) {
        // damped: D <- (1 - kDamp) D_new + kDamp D
        MESS_TRY(density_from_projector(st, s, st->W2));
        MESS_TRY(axpby(s, nn, 1.0 - kDamp, st->W2, kDamp, st->D, st->D));
    } else {
        MESS_TRY(density_from_projector(st, s, st->D));
    }
    (void)M;
    return MESS_OK;
}

// ------------------------------------------------ direct minimisation
//
// E(Z) over an unconstrained square trial matrix Z: Z = Q R (QR
// decomposition), C = X Q with the Loewdin X = S^{-1/2} (so C^T S C = 1,
// the orthonormality constraint), D = 2 C_occ C_occ^T, E as in the SCF step.
// Gradient: dE/dC_occ = 4 F C_occ; Qbar = X^T Cbar; with B = Qbar^T Q,
// dE/dZ = Q tril(B^T - B, -1) R^{-T}.  Q and R come from the Cholesky
// factor of Z^T Z (R upper with positive diagonal, Q = Z R^{-1}); E and its
// gradient do not depend on the sign convention of the QR factors.

__global__ void k_fill_int(int *__restrict__ p, int v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// In place: A (n x n, symmetric positive definite) -> upper Cholesky factor
// R with A = R^T R (the strict lower triangle set to zero); flag = 1 if a
// pivot is not positive.  One workgroup.
__global__ void __launch_bounds__(1024) k_chol_upper(int n, double *__restrict__ A, int *__restrict__ flag) {
    for (int k = 0; k < n; ++k) {
        __syncthreads();
        const double akk = A[(int64_t)k * n + k];
        if (!(akk > 0.0)) {
            if (threadIdx.x == 0) *flag = 1;
            return;
        }
        const double r = sqrt(akk), ir = 1.0 / r;
        __syncthreads();
        for (int j = k + threadIdx.x; j < n; j += blockDim.x) A[(int64_t)k * n + j] = j == k ? r : A[(int64_t)k * n + j] * ir;
        __syncthreads();
        // trailing update of the upper triangle: A[i][j] -= R[k][i] R[k][j], k < i <= j
        const int m = n - k - 1;
        for (int64_t t = threadIdx.x; t < (int64_t)m * m; t += blockDim.x) {
            const int i = k + 1 + (int)(t / m), j = k + 1 + (int)(t % m);
            if (j >= i) A[(int64_t)i * n + j] -= A[(int64_t)k * n + i] * A[(int64_t)k * n + j];
        }
    }
    __syncthreads();
    for (int64_t t = threadIdx.x; t < (int64_t)n * n; t += blockDim.x)
        if (t / n > t % n) A[t] = 0.0;
}

// Row-wise triangular solves with the upper factor R (n x n), one thread per
// row: trans = 0: X R = B (X = B R^{-1}); trans = 1: X R^T = B.
__global__ void k_trsm_rows(int n, const double *__restrict__ R, const double *__restrict__ Bm, double *__restrict__ X,
                            int trans) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double *b = Bm + (int64_t)i * n;
    double *x = X + (int64_t)i * n;
    if (!trans) {
        for (int j = 0; j < n; ++j) {
            double s = b[j];
            for (int k = 0; k < j; ++k) s -= x[k] * R[(int64_t)k * n + j];
            x[j] = s / R[(int64_t)j * n + j];
        }
    } else {
        for (int j = n - 1; j >= 0; --j) {
            double s = b[j];
            for (int k = j + 1; k < n; ++k) s -= R[(int64_t)j * n + k] * x[k];
            x[j] = s / R[(int64_t)j * n + j];
        }
    }
}

// W = tril(B^T - B, -1) for B with rows >= nb zero (B stored nb x n).
__global__ void k_tril_skew(int n, int nb, const double *__restrict__ Bm, double *__restrict__ W) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < (int64_t)n * n;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(t / n), j = (int)(t % n);
        double v = 0.0;
        if (i > j) v = (j < nb ? Bm[(int64_t)j * n + i] : 0.0) - (i < nb ? Bm[(int64_t)i * n + j] : 0.0);
        W[t] = v;
    }
}

// Adam step on Z with gradient g (bias-corrected; b1 = 0.9, b2 = 0.999, eps = 1e-8).
__global__ void k_adam(int64_t n, double lr, double c1, double c2, const double *__restrict__ g, double *__restrict__ m,
                       double *__restrict__ v, double *__restrict__ Z) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const double gt = g[t];
        const double mt = 0.9 * m[t] + 0.1 * gt;
        const double vt = 0.999 * v[t] + 0.001 * gt * gt;
        m[t] = mt;
        v[t] = vt;
        Z[t] -= lr * (mt / c1) / (sqrt(vt / c2) + 1e-8);
    }
}

__global__ void k_set_identity(int n, double *__restrict__ A) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < (int64_t)n * n;
         t += (int64_t)gridDim.x * blockDim.x)
        A[t] = (t / n == t % n) ? 1.0 : 0.0;
}

static int dmin_buffers(mess_scf *st, hipStream_t s) {
    const int N = st->N;
    const int64_t nn = (int64_t)N * N;
    if (!st->Zt) {
        for (double **p : {&st->Zt, &st->Qf, &st->Rf, &st->Am, &st->Av, &st->Gz})
            MESS_HIP(hipMalloc(p, sizeof(double) * std::max<int64_t>(nn, 16)));
        hipLaunchKernelGGL(k_set_identity, dim3(grid1(nn)), dim3(256), 0, s, N, st->Zt);
        MESS_TRY(zero_async(st->Am, nn, s));
        MESS_TRY(zero_async(st->Av, nn, s));
        st->dmin_t = 0;
    }
    return MESS_OK;
}

// E(Z) and dE/dZ (into Gz) for the trial matrix Zin (device N x N).
static int dmin_eval(mess_scf *st, const double *Zin, double *energy, double *gmax, hipStream_t s) {
    mess_basis *B = st->basis;
    const int N = st->N, n = B->nocc;
    const int64_t nn = (int64_t)N * N;
    const unsigned gew = (unsigned)grid1(nn);
    MESS_TRY(dmin_buffers(st, s));
    // QR of Z through the Cholesky factor of Z^T Z
    MESS_TRY(gemm(s, true, false, N, N, N, 1.0, Zin, N, Zin, N, 0.0, st->Rf, N));
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, s, &st->sc->flag, 0);
    hipLaunchKernelGGL(k_chol_upper, dim3(1), dim3(1024), 0, s, N, st->Rf, &st->sc->flag);
    hipLaunchKernelGGL(k_trsm_rows, dim3((N + 63) / 64), dim3(64), 0, s, N, st->Rf, Zin, st->Qf, 0);
    MESS_LAUNCH_CHECK();
    // C = X Q (in W1), D = 2 C_occ C_occ^T
    MESS_TRY(gemm(s, false, false, N, N, N, 1.0, st->X, N, st->Qf, N, 0.0, st->W1, N));
    MESS_TRY(gemm(s, false, true, N, N, n, 2.0, st->W1, N, st->W1, N, 0.0, st->D, N));
    // F and E
    MESS_TRY(scf_jk(st, st->D, st->Gj, st->Gk, st->opts.prec, st->opts.schwarz_tol, s));
    hipLaunchKernelGGL(k_fock, dim3(kRedBlocks), dim3(256), 0, s, N, st->H, st->Gj, st->Gk, (const double *)nullptr,
                       st->D, st->F, st->partial);
    hipLaunchKernelGGL(k_finish_energy, dim3(1), dim3(256), 0, s, kRedBlocks, st->partial, B->enuc,
                       (const double *)nullptr, st->sc);
    MESS_LAUNCH_CHECK();
    // Cbar = 4 F C_occ (N x n, in W2, leading dimension N); Qbar = X^T Cbar (W3)
    MESS_TRY(gemm(s, false, false, N, n, N, 4.0, st->F, N, st->W1, N, 0.0, st->W2, N));
    MESS_TRY(gemm(s, true, false, N, n, N, 1.0, st->X, N, st->W2, N, 0.0, st->W3, N));
    // B = Qbar^T Q (n x N, in P); W = tril(B^T - B, -1) (P2); Gz = (Q W) R^{-T}
    MESS_TRY(gemm(s, true, false, n, N, N, 1.0, st->W3, N, st->Qf, N, 0.0, st->P, N));
    hipLaunchKernelGGL(k_tril_skew, dim3(gew), dim3(256), 0, s, N, n, st->P, st->P2);
    MESS_TRY(gemm(s, false, false, N, N, N, 1.0, st->Qf, N, st->P2, N, 0.0, st->W1, N));
    hipLaunchKernelGGL(k_trsm_rows, dim3((N + 63) / 64), dim3(64), 0, s, N, st->Rf, st->W1, st->Gz, 1);
    hipLaunchKernelGGL(k_maxabs_to, dim3(1), dim3(1024), 0, s, nn, st->Gz, &st->sc->dmax);
    MESS_LAUNCH_CHECK();
    ScfScalars h;
    MESS_HIP(hipMemcpyAsync(&h, st->sc, sizeof(ScfScalars), hipMemcpyDeviceToHost, s));
    MESS_HIP(hipStreamSynchronize(s));
    if (h.flag) {
        set_error("mess_dmin_step: the trial matrix became singular (Z^T Z not positive definite)");
        return MESS_E_NUMERIC;
    }
    if (!std::isfinite(h.energy) || !std::isfinite(h.dmax)) {
        set_error("mess_dmin_step: non-finite energy or gradient");
        return MESS_E_NUMERIC;
    }
    if (energy) *energy = h.energy;
    if (gmax) *gmax = h.dmax;
    return MESS_OK;
}

static int dmin_step_impl(mess_scf *st, double lr, double *energy, double *gmax, hipStream_t s) {
    const int64_t nn = (int64_t)st->N * st->N;
    const unsigned gew = (unsigned)grid1(nn);
    MESS_TRY(dmin_buffers(st, s));
    MESS_TRY(dmin_eval(st, st->Zt, energy, gmax, s));
    // Adam update of Z
    st->dmin_t += 1;
    const double c1 = 1.0 - std::pow(0.9, st->dmin_t), c2 = 1.0 - std::pow(0.999, st->dmin_t);
    hipLaunchKernelGGL(k_adam, dim3(gew), dim3(256), 0, s, nn, lr, c1, c2, st->Gz, st->Am, st->Av, st->Zt);
    MESS_LAUNCH_CHECK();
    return MESS_OK;
}

}  // namespace mess

using namespace mess;

extern "C" {

int mess_scf_create(const mess_basis *basis, const mess_scf_opts *opts, const double *D0, mess_scf **out) {
    if (!basis || !opts || !out) {
        set_error("mess_scf_create: NULL basis, options or output");
        return MESS_E_ARG;
    }
    *out = nullptr;
    if (basis->n_mol != 1) {
        set_error("mess_scf_create: the basis holds a batch of %d molecules; use mess_batch_scf_create",
                  basis->n_mol);
        return MESS_E_ARG;
    }
    if (basis->nelec % 2) {
        set_error("mess_scf_create: %d electrons; only closed-shell (even) systems are supported", basis->nelec);
        return MESS_E_UNSUPPORTED;
    }
    if (opts->jk_mode != MESS_JK_DIRECT && opts->jk_mode != MESS_JK_STORED &&
        opts->jk_mode != MESS_JK_DETERMINISTIC) {
        set_error("mess_scf_create: unknown J/K mode %d", opts->jk_mode);
        return MESS_E_UNSUPPORTED;
    }
    if (opts->prec != MESS_FP64 && opts->prec != MESS_FP32) {
        set_error("mess_scf_create: unknown precision %d", opts->prec);
        return MESS_E_UNSUPPORTED;
    }
    if (opts->xc != MESS_XC_HF && opts->xc != MESS_XC_LDA_X && opts->xc != MESS_XC_PBE) {
        set_error("mess_scf_create: unknown exchange form %d", opts->xc);
        return MESS_E_UNSUPPORTED;
    }
    if (opts->xc != MESS_XC_HF && opts->prec != MESS_FP64) {
        set_error("mess_scf_create: LDA and PBE run in FP64 only");
        return MESS_E_UNSUPPORTED;
    }
    if (opts->diis_size < 0 || opts->diis_size > kMaxDiis || !(opts->conv_tol >= 0.0)) {
        set_error("mess_scf_create: diis_size must be 0..%d and conv_tol >= 0", kMaxDiis);
        return MESS_E_ARG;
    }
    auto *st = new mess_scf();
    st->basis = const_cast<mess_basis *>(basis);
    st->opts = *opts;
    int rc = scf_create_impl(st, D0);
    if (rc != MESS_OK) {
        free_scf(st);
        return rc;
    }
    *out = st;
    return MESS_OK;
}

int mess_scf_step(mess_scf *scf, double *energy, double *delta_e, double *resid, int32_t *converged,
                  mess_stream stream) {
    if (!scf) {
        set_error("mess_scf_step: NULL handle");
        return MESS_E_ARG;
    }
    return scf_step_impl(scf, energy, delta_e, resid, converged, static_cast<hipStream_t>(stream));
}

int mess_scf_gradient(const mess_scf *scf, double *grad, mess_stream stream) {
    if (!scf || !grad) {
        set_error("mess_scf_gradient: NULL argument");
        return MESS_E_ARG;
    }
    if (scf->opts.xc != MESS_XC_HF) {
        set_error("mess_scf_gradient: the gradient is built for Hartree-Fock exchange");
        return MESS_E_UNSUPPORTED;
    }
    return mess_hf_gradient(scf->basis, scf->D, scf->F, scf->opts.schwarz_tol, grad, stream);
}

int mess_scf_guard(const mess_scf *scf, int32_t *stage, int32_t *rises) {
    if (!scf) {
        set_error("mess_scf_guard: NULL handle");
        return MESS_E_ARG;
    }
    if (stage) *stage = scf->stage;
    if (rises) *rises = scf->rises;
    return MESS_OK;
}

int mess_scf_density(const mess_scf *scf, double *D, mess_stream stream) {
    if (!scf || !D) {
        set_error("mess_scf_density: NULL argument");
        return MESS_E_ARG;
    }
    MESS_HIP(hipMemcpyAsync(D, scf->D, sizeof(double) * scf->N * scf->N, hipMemcpyDeviceToDevice,
                            static_cast<hipStream_t>(stream)));
    return MESS_OK;
}

int mess_scf_fock(const mess_scf *scf, double *F, mess_stream stream) {
    if (!scf || !F) {
        set_error("mess_scf_fock: NULL argument");
        return MESS_E_ARG;
    }
    MESS_HIP(hipMemcpyAsync(F, scf->F, sizeof(double) * scf->N * scf->N, hipMemcpyDeviceToDevice,
                            static_cast<hipStream_t>(stream)));
    return MESS_OK;
}

void mess_scf_destroy(mess_scf *scf) { free_scf(scf); }

int mess_dmin_step(mess_scf *scf, double lr, double *energy, double *grad_max, mess_stream stream) {
    if (!scf) {
        set_error("mess_dmin_step: NULL handle");
        return MESS_E_ARG;
    }
    if (!(lr > 0.0) || !std::isfinite(lr)) {
        set_error("mess_dmin_step: learning rate must be positive and finite");
        return MESS_E_ARG;
    }
    if (scf->M != scf->N) {
        set_error("mess_dmin_step: the overlap needed the canonical orthogonaliser (%d of %d functions kept); "
                  "direct minimisation needs the Loewdin S^-1/2", scf->M, scf->N);
        return MESS_E_UNSUPPORTED;
    }
    if (scf->opts.xc != MESS_XC_HF) {
        set_error("mess_dmin_step: only the Hartree-Fock energy is minimised directly");
        return MESS_E_UNSUPPORTED;
    }
    return dmin_step_impl(scf, lr, energy, grad_max, static_cast<hipStream_t>(stream));
}

int mess_dmin_eval(mess_scf *scf, const double *Z, double *energy, double *G, mess_stream stream) {
    if (!scf || !Z) {
        set_error("mess_dmin_eval: NULL handle or trial matrix");
        return MESS_E_ARG;
    }
    if (scf->M != scf->N || scf->opts.xc != MESS_XC_HF) {
        set_error("mess_dmin_eval: needs the Loewdin S^-1/2 and the Hartree-Fock energy");
        return MESS_E_UNSUPPORTED;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    MESS_TRY(dmin_eval(scf, Z, energy, nullptr, s));
    if (G)
        MESS_HIP(hipMemcpyAsync(G, scf->Gz, sizeof(double) * scf->N * scf->N, hipMemcpyDeviceToDevice, s));
    MESS_HIP(hipStreamSynchronize(s));
    return MESS_OK;
}

int mess_dmin_trial(const mess_scf *scf, double *Z, mess_stream stream) {
    if (!scf || !Z) {
        set_error("mess_dmin_trial: NULL argument");
        return MESS_E_ARG;
    }
    if (!scf->Zt) {
        set_error("mess_dmin_trial: no direct-minimisation step has run on this handle");
        return MESS_E_ARG;
    }
    MESS_HIP(hipMemcpyAsync(Z, scf->Zt, sizeof(double) * scf->N * scf->N, hipMemcpyDeviceToDevice,
                            static_cast<hipStream_t>(stream)));
    return MESS_OK;
}

}  // extern "C"
