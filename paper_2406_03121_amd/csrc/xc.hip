// LDA exchange on an atom-centred molecular grid (paper section 5 names the
// local density approximation as the exchange-correlation choice of its
// batched example; functional and grid are this library's readings):
//
//   Dirac-Slater exchange  e_x(rho) = -C_x rho^(4/3),  C_x = (3/4)(3/pi)^(1/3),
//   v_x = de_x/drho = -(3/pi)^(1/3) rho^(1/3)  (points with rho <= 0 add nothing);
//   rho_g = sum_{mu nu} Phi_{g mu} D_{mu nu} Phi_{g nu},
//   E_x = sum_g w_g e_x(rho_g),  V_x = Phi^T diag(w v_x) Phi.
//
// Grid per atom: 75 second-kind Gauss-Chebyshev radial nodes
// x_i = cos(i pi / 76) mapped by r = (1 + x)/(1 - x) bohr, times a product
// angular rule of 17 Gauss-Legendre nodes in cos(theta) and 34 equally
// spaced azimuths; Becke fuzzy-cell weights (three smoothing iterations, no
// size adjustment).  Points are ordered atom, radial node, theta, azimuth.
//
// Device layout: the grid as [G][4] (x, y, z, w) and the basis values
// transposed, PhiT[mu][g] with G (the point count rounded up to 64)
// contiguous, so that the basis-value kernel writes coalesced rows and both
// contractions stream G-contiguous tiles.  Both are built once per basis.
// Per density: one kernel forms U = D PhiT on a 64-point tile, chunk by
// chunk of 64 rows, and reduces rho_g = sum_nu PhiT[nu][g] U[nu][g] in the
// same pass (2 N^2 flops per point), then the weights f_g = w_g v_x(rho_g);
// a second kernel forms V_x = PhiT diag(f) PhiT^T on 64 x 64 tiles of the
// upper block triangle over chunks of points, adding tile partials into
// V_x with FP64 atomics (2 N^2 flops per point in all).
//
// PBE exchange-correlation (the generalised-gradient functional the paper
// selects for its DFT examples, section 5), closed shell, on the same grid:
//   f(rho, sigma) = rho eps_x^unif F_x(s) + rho (eps_c^PW92(r_s) + H(r_s, t)),
//   sigma = |grad rho|^2, grad rho = 2 sum_{mu nu} D_{mu nu} phi_mu grad phi_nu,
//   E_xc = sum_g w_g f_g,
//   V_xc[mu][nu] = sum_g w_g [f_rho phi_mu phi_nu
//                             + 2 f_sigma grad rho . (phi_mu grad phi_nu + grad phi_mu phi_nu)],
// with the partial derivatives f_rho, f_sigma written out analytically
// (pbe_point); points with rho < 1e-10 add nothing.  The basis gradients
// dPhiT[k][mu][g] (k = x, y, z) are built on the first PBE call.  Per
// density: U = D PhiT per 64-point tile reduced against PhiT and the three
// dPhiT (rho and grad rho in one pass, 2 N^2 + 6 N flops per point), the
// functional per point, and V_xc = PhiT Z^T + Z PhiT^T with
// Z[nu][g] = w (f_rho/2 phi_nu + 2 f_sigma grad rho . grad phi_nu) formed
// while the tiles are staged (all tile pairs, 2 N^2 flops per point).
#include <algorithm>
#include <cmath>
#include <vector>

#include "eri_hgp.hpp"
#include "mess_internal.hpp"

namespace mess {

constexpr int kNRad = 75, kNTheta = 17, kNPhi = 34, kNAng = kNTheta * kNPhi;
constexpr int kPtsPerAtom = kNRad * kNAng;
constexpr int kXT = 64;      // tile edge of both contractions
constexpr int kXK = 16;      // contraction step staged in LDS
constexpr int kVChunk = 32768;  // points per V_x partial

struct XcShell {
    double x, y, z;
    int l, prim0, nprim, bf0;
};

struct XcGrid {
    int64_t npts = 0, G = 0;
    int nbf = 0, nrho_blocks = 0;
    double *dphiT = nullptr;  // [3][nbf][G] basis gradients (PBE only)
    double *grad = nullptr;   // [3][G] grad rho (PBE)
    double *hv = nullptr;     // [3][G] 2 w f_sigma grad rho (PBE)
    double *xyzw = nullptr;   // [G][4]
    double *phiT = nullptr;   // [nbf][G]
    double *f = nullptr;      // [G] w_g v_x(rho_g)
    double *rho = nullptr;    // [G]
    double *epart = nullptr;  // [nrho_blocks] partial sums of w_g e_x
    double *ex = nullptr;     // [1] E_x of the last build
    double *Vacc = nullptr;   // [nbf][nbf] accumulation of the upper block triangle
};

void free_xc(mess_basis *B) {
    XcGrid *X = static_cast<XcGrid *>(B->xc);
    if (!X) return;
    for (double *p : {X->xyzw, X->phiT, X->f, X->rho, X->epart, X->ex, X->Vacc, X->dphiT, X->grad, X->hv}) hipFree(p);
    delete X;
    B->xc = nullptr;
}

// ------------------------------------------------------------ quadrature

// Gauss-Legendre nodes (ascending) and weights on [-1, 1]: Newton's method on
// P_n from the three-term recurrence, started at cos(pi (i - 1/4)/(n + 1/2)).
static void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 1; i <= n; ++i) {
        double z = std::cos(M_PI * (i - 0.25) / (n + 0.5)), dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
        }
        x[n - i] = z;  // z decreases with i
        w[n - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// Becke cell function s(mu) = (1 - f(f(f(mu))))/2, f(x) = (3x - x^3)/2.
__device__ __forceinline__ double becke_s(double mu) {
    double f = mu;
#pragma unroll
    for (int k = 0; k < 3; ++k) f = 1.5 * f - 0.5 * f * f * f;
    return 0.5 * (1.0 - f);
}

// One thread per point: position and weight (radial x angular x Becke).
__global__ void k_grid(int nat, const double *__restrict__ xyz, const double *__restrict__ rad,
                       const double *__restrict__ ang, int64_t npts, int64_t G, double *__restrict__ xyzw) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= G) return;
    if (g >= npts) {
        xyzw[4 * g] = xyzw[4 * g + 1] = xyzw[4 * g + 2] = xyzw[4 * g + 3] = 0.0;
        return;
    }
    const int a = (int)(g / kPtsPerAtom);
    const int rest = (int)(g % kPtsPerAtom);
    const int ir = rest / kNAng, ia = rest % kNAng;
    const double r = rad[2 * ir], wr = rad[2 * ir + 1];
    const double px = xyz[3 * a] + r * ang[4 * ia], py = xyz[3 * a + 1] + r * ang[4 * ia + 1],
                 pz = xyz[3 * a + 2] + r * ang[4 * ia + 2];
    double Pown = 0.0, Psum = 0.0;
    for (int c = 0; c < nat; ++c) {
        const double dcx = px - xyz[3 * c], dcy = py - xyz[3 * c + 1], dcz = pz - xyz[3 * c + 2];
        const double dc = sqrt(dcx * dcx + dcy * dcy + dcz * dcz);
        double P = 1.0;
        for (int b = 0; b < nat; ++b) {
            if (b == c) continue;
            const double dbx = px - xyz[3 * b], dby = py - xyz[3 * b + 1], dbz = pz - xyz[3 * b + 2];
            const double db = sqrt(dbx * dbx + dby * dby + dbz * dbz);
            const double ex = xyz[3 * c] - xyz[3 * b], ey = xyz[3 * c + 1] - xyz[3 * b + 1],
                         ez = xyz[3 * c + 2] - xyz[3 * b + 2];
            const double R = sqrt(ex * ex + ey * ey + ez * ez);
            P *= becke_s((dc - db) / R);
        }
        Psum += P;
        if (c == a) Pown = P;
    }
    xyzw[4 * g] = px;
    xyzw[4 * g + 1] = py;
    xyzw[4 * g + 2] = pz;
    xyzw[4 * g + 3] = wr * ang[4 * ia + 3] * (Pown / Psum);
}

// PhiT[mu][g]: one thread per point, loop over shells.  Contraction
// coefficients are those of the (l,0,0) component; mixed d components carry
// the factor sqrt(3).
__global__ void k_basis_values(int nsh, const XcShell *__restrict__ sh, const double *__restrict__ alpha,
                               const double *__restrict__ ct, int64_t npts, int64_t G,
                               const double *__restrict__ xyzw, double *__restrict__ phiT) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= G) return;
    const bool live = g < npts;
    const double px = xyzw[4 * g], py = xyzw[4 * g + 1], pz = xyzw[4 * g + 2];
    for (int s = 0; s < nsh; ++s) {
        const XcShell S = sh[s];
        const double dx = px - S.x, dy = py - S.y, dz = pz - S.z;
        const double r2 = dx * dx + dy * dy + dz * dz;
        double rad = 0.0;
        if (live)
            for (int p = 0; p < S.nprim; ++p) {
                const double e = alpha[S.prim0 + p] * r2;
                if (e < 745.0) rad += ct[S.prim0 + p] * exp(-e);
            }
        double *o = phiT + (int64_t)S.bf0 * G + g;
        if (S.l == 0) {
            o[0] = rad;
        } else if (S.l == 1) {
            o[0] = dx * rad;
            o[G] = dy * rad;
            o[2 * G] = dz * rad;
        } else {
            // xx, xy, xz, yy, yz, zz
            o[0] = dx * dx * rad;
            o[G] = kSqrt3 * dx * dy * rad;
            o[2 * G] = kSqrt3 * dx * dz * rad;
            o[3 * G] = dy * dy * rad;
            o[4 * G] = kSqrt3 * dy * dz * rad;
            o[5 * G] = dz * dz * rad;
        }
    }
}

// dPhiT[k][mu][g] = d phi_mu / d r_k at point g: one thread per point, loop
// over shells; for x^a y^b z^c R(r^2), R = sum c_p e^{-alpha_p r^2},
// d/dx = a x^(a-1) y^b z^c R - 2 x (x^a y^b z^c) sum c_p alpha_p e^{-alpha_p r^2}.
__global__ void k_basis_grad(int nsh, const XcShell *__restrict__ sh, const double *__restrict__ alpha,
                             const double *__restrict__ ct, int64_t npts, int64_t G, int nbf,
                             const double *__restrict__ xyzw, double *__restrict__ dphiT) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= G) return;
    const bool live = g < npts;
    const double px = xyzw[4 * g], py = xyzw[4 * g + 1], pz = xyzw[4 * g + 2];
    const int64_t plane = (int64_t)nbf * G;
    for (int s = 0; s < nsh; ++s) {
        const XcShell S = sh[s];
        const double d[3] = {px - S.x, py - S.y, pz - S.z};
        const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        double rad = 0.0, drad = 0.0;
        if (live)
            for (int p = 0; p < S.nprim; ++p) {
                const double a = alpha[S.prim0 + p], e = a * r2;
                if (e < 745.0) {
                    const double t = ct[S.prim0 + p] * exp(-e);
                    rad += t;
                    drad += a * t;
                }
            }
        const int nc = (S.l + 1) * (S.l + 2) / 2;
        for (int c = 0; c < nc; ++c) {
            // component exponents in the order x-major (xx, xy, xz, yy, yz, zz)
            int e[3];
            if (S.l == 0) {
                e[0] = e[1] = e[2] = 0;
            } else if (S.l == 1) {
                e[0] = c == 0;
                e[1] = c == 1;
                e[2] = c == 2;
            } else {
                const int tab[6][3] = {{2, 0, 0}, {1, 1, 0}, {1, 0, 1}, {0, 2, 0}, {0, 1, 1}, {0, 0, 2}};
                e[0] = tab[c][0];
                e[1] = tab[c][1];
                e[2] = tab[c][2];
            }
            const double sc = (S.l == 2 && (c == 1 || c == 2 || c == 4)) ? kSqrt3 : 1.0;
            double mono = 1.0;
            for (int k = 0; k < 3; ++k)
                for (int q = 0; q < e[k]; ++q) mono *= d[k];
            for (int k = 0; k < 3; ++k) {
                double lower = 0.0;
                if (e[k] > 0) {
                    lower = e[k];
                    for (int j = 0; j < 3; ++j)
                        for (int q = 0; q < e[j] - (j == k); ++q) lower *= d[j];
                }
                dphiT[k * plane + (int64_t)(S.bf0 + c) * G + g] = sc * (lower * rad - 2.0 * d[k] * mono * drad);
            }
        }
    }
}

// ------------------------------------------------------------ per density

__device__ __forceinline__ void exchange_terms(double rho, double &ex, double &vx) {
    constexpr double kCx = 0.73855876638202240587;   // (3/4)(3/pi)^(1/3)
    constexpr double kVx = 0.98474502184269654116;   // (3/pi)^(1/3)
    if (rho > 0.0) {
        const double c = cbrt(rho);
        ex = -kCx * rho * c;
        vx = -kVx * c;
    } else {
        ex = 0.0;
        vx = 0.0;
    }
}

// rho over a 64-point tile: U = D PhiT[:, tile] by 64-row chunks (4 x 4
// register blocking per thread, K staged through LDS), rho_g accumulated
// from the chunk and PhiT; then f_g and the block's partial sum of w e_x.
__global__ void __launch_bounds__(256) k_lda_rho(int N, int64_t G, const double *__restrict__ D,
                                                 const double *__restrict__ phiT, const double *__restrict__ xyzw,
                                                 double *__restrict__ rho_out, double *__restrict__ f,
                                                 double *__restrict__ epart) {
    __shared__ double As[kXK][kXT + 1];
    __shared__ double Bs[kXK][kXT + 1];
    __shared__ double red[16][kXT + 1];
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const int64_t g0 = (int64_t)blockIdx.x * kXT;
    double part[4] = {0.0, 0.0, 0.0, 0.0};
    for (int nu0 = 0; nu0 < N; nu0 += kXT) {
        double acc[4][4] = {};
        for (int k0 = 0; k0 < N; k0 += kXK) {
            for (int t = threadIdx.x; t < kXK * kXT; t += 256) {
                const int kk = t % kXK, mm = t / kXK;  // D rows, K contiguous
                const int r = nu0 + mm, k = k0 + kk;
                As[kk][mm] = (r < N && k < N) ? D[(int64_t)r * N + k] : 0.0;
            }
            for (int t = threadIdx.x; t < kXK * kXT; t += 256) {
                const int kk = t / kXT, nn = t % kXT;  // PhiT rows, points contiguous
                const int k = k0 + kk;
                Bs[kk][nn] = k < N ? phiT[(int64_t)k * G + g0 + nn] : 0.0;
            }
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < kXK; ++kk) {
                double a[4], b[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
                for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx + 16 * j];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
            }
            __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int nu = nu0 + ty + 16 * i;
            if (nu >= N) continue;
#pragma unroll
            for (int j = 0; j < 4; ++j) part[j] = fma(phiT[(int64_t)nu * G + g0 + tx + 16 * j], acc[i][j], part[j]);
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) red[ty][tx + 16 * j] = part[j];
    __syncthreads();
    double e = 0.0;
    if (threadIdx.x < kXT) {
        const int c = threadIdx.x;
        double r = 0.0;
        for (int k = 0; k < 16; ++k) r += red[k][c];
        const int64_t g = g0 + c;
        const double w = xyzw[4 * g + 3];
        double ex, vx;
        exchange_terms(r, ex, vx);
        rho_out[g] = r;
        f[g] = w * vx;
        e = w * ex;
    }
    __syncthreads();
    // block sum of w e_x (fixed order)
    if (threadIdx.x < kXT) red[0][threadIdx.x] = e;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int c = 0; c < kXT; ++c) s += red[0][c];
        epart[blockIdx.x] = s;
    }
}

__global__ void __launch_bounds__(256) k_sum_partials(int n, const double *__restrict__ part, double *__restrict__ out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

// Vacc[mu][nu] += sum_{g in chunk} PhiT[mu][g] f_g PhiT[nu][g] for the tile
// pair (bi <= bj) given by blockIdx.y; blockIdx.x is the point chunk.
__global__ void __launch_bounds__(256) k_lda_v(int N, int64_t G, int nblk, const double *__restrict__ phiT,
                                               const double *__restrict__ f, double *__restrict__ Vacc) {
    __shared__ double As[kXK][kXT + 1];
    __shared__ double Bs[kXK][kXT + 1];
    int bi = 0, rem = blockIdx.y;
    while (rem >= nblk - bi) {
        rem -= nblk - bi;
        ++bi;
    }
    const int bj = bi + rem;
    const int row0 = bi * kXT, col0 = bj * kXT;
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const int64_t gs = (int64_t)blockIdx.x * kVChunk;
    const int64_t ge = gs + kVChunk < G ? gs + kVChunk : G;
    double acc[4][4] = {};
    for (int64_t k0 = gs; k0 < ge; k0 += kXK) {
        for (int t = threadIdx.x; t < kXK * kXT; t += 256) {
            const int kk = t % kXK, mm = t / kXK;
            const int r = row0 + mm;
            As[kk][mm] = r < N ? phiT[(int64_t)r * G + k0 + kk] : 0.0;
        }
        for (int t = threadIdx.x; t < kXK * kXT; t += 256) {
            const int kk = t % kXK, nn = t / kXK;
            const int c = col0 + nn;
            Bs[kk][nn] = c < N ? f[k0 + kk] * phiT[(int64_t)c * G + k0 + kk] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kXK; ++kk) {
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx + 16 * j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = row0 + ty + 16 * i;
        if (r >= N) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int c = col0 + tx + 16 * j;
            if (c < N) unsafeAtomicAdd(&Vacc[(int64_t)r * N + c], acc[i][j]);
        }
    }
}

// V[i][j] from the upper triangle of Vacc (the upper block triangle was
// accumulated; inside a diagonal block only i <= j is taken, so V is exactly
// symmetric).
__global__ void k_lda_mirror(int N, const double *__restrict__ Vacc, double *__restrict__ V) {
    const int64_t NN = (int64_t)N * N;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < NN; idx += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(idx / N), j = (int)(idx % N);
        V[idx] = (i <= j) ? Vacc[idx] : Vacc[(int64_t)j * N + i];
    }
}

// ------------------------------------------------------------------ PBE

constexpr double kRhoMin = 1e-10;

// f = rho eps_x^unif F_x + rho (eps_c + H) and its partial derivatives in
// rho and sigma (closed shell, Hartree atomic units).
//   exchange: s^2 = c_s sigma rho^(-8/3), c_s = 1 / (4 (3 pi^2)^(2/3)),
//     F_x = 1 + kappa - kappa / (1 + mu s^2 / kappa);
//   correlation: Perdew-Wang eps_c(r_s), r_s = (3 / (4 pi rho))^(1/3);
//     t^2 = c_t sigma rho^(-7/3), c_t = pi / (16 (3 pi^2)^(1/3));
//     H = gamma ln(1 + (beta/gamma) t^2 R(A t^2)), R(y) = (1 + y)/(1 + y + y^2),
//     A = (beta/gamma) / (exp(-eps_c/gamma) - 1).
__device__ __forceinline__ void pbe_point(double rho, double sigma, double &f, double &fr, double &fs) {
    if (!(rho >= kRhoMin)) {
        f = fr = fs = 0.0;
        return;
    }
    constexpr double kKappa = 0.804, kBeta = 0.06672455060314922;
    constexpr double kMu = kBeta * M_PI * M_PI / 3.0;
    constexpr double kGamma = 0.031090690869654895;  // (1 - ln 2) / pi^2
    constexpr double kA = 0.031091, kA1 = 0.21370, kB1 = 7.5957, kB2 = 3.5876, kB3 = 1.6382, kB4 = 0.49294;
    constexpr double kCx = -0.73855876638202240587;  // -(3/4)(3/pi)^(1/3)
    constexpr double kCs = 0.026121172985233599;     // 1 / (4 (3 pi^2)^(2/3))
    constexpr double kCt = 0.063468206097703704;     // pi / (16 (3 pi^2)^(1/3))
    constexpr double kRs = 0.62035049089940001667;   // (3 / (4 pi))^(1/3)
    const double r13 = cbrt(rho), r43 = rho * r13;
    const double ir43 = 1.0 / r43, ir83 = ir43 * ir43;
    // exchange
    const double x = kCs * sigma * ir83;
    const double den = 1.0 + kMu * x / kKappa;
    const double Fx = 1.0 + kKappa - kKappa / den;
    const double Fxp = kMu / (den * den);
    const double ex = kCx * r43 * Fx;
    const double exr = kCx * r13 * ((4.0 / 3.0) * Fx - (8.0 / 3.0) * x * Fxp);
    const double exs = kCx * Fxp * kCs * ir43;
    // Perdew-Wang correlation of the uniform gas
    const double rs = kRs / r13, sq = sqrt(rs);
    const double Q = 2.0 * kA * (kB1 * sq + kB2 * rs + kB3 * rs * sq + kB4 * rs * rs);
    const double Qp = 2.0 * kA * (0.5 * kB1 / sq + kB2 + 1.5 * kB3 * sq + 2.0 * kB4 * rs);
    const double Lg = log1p(1.0 / Q);
    const double ec = -2.0 * kA * (1.0 + kA1 * rs) * Lg;
    const double dec = -2.0 * kA * kA1 * Lg + 2.0 * kA * (1.0 + kA1 * rs) * Qp / (Q * Q + Q);
    // gradient correction
    const double u = kCt * sigma * ir43 / rho;  // t^2
    const double E1 = expm1(-ec / kGamma);
    const double Ap = (kBeta / kGamma) / E1;
    const double y = Ap * u, d2 = 1.0 + y + y * y;
    const double R = (1.0 + y) / d2, Rp = -y * (2.0 + y) / (d2 * d2);
    const double Nn = (kBeta / kGamma) * u * R;
    const double H = kGamma * log1p(Nn);
    const double dHdN = kGamma / (1.0 + Nn);
    const double dHdu = dHdN * (kBeta / kGamma) * (R + y * Rp);
    const double dHdec = dHdN * (kBeta / kGamma) * u * u * Rp * (Ap * Ap * (E1 + 1.0) / kBeta);
    f = ex + rho * (ec + H);
    fr = exr + ec + H - (rs / 3.0) * dec * (1.0 + dHdec) - (7.0 / 3.0) * u * dHdu;
    fs = exs + dHdu * kCt * ir43;
}

// rho and grad rho over a 64-point tile: U = D PhiT[:, tile] by 64-row
// chunks as in k_lda_rho, reduced against PhiT (rho) and the three basis
// gradient planes (grad rho = 2 sum_nu dPhiT[k][nu][g] U[nu][g]).
__global__ void __launch_bounds__(256) k_gga_rho(int N, int64_t G, const double *__restrict__ D,
                                                 const double *__restrict__ phiT, const double *__restrict__ dphiT,
                                                 double *__restrict__ rho_out, double *__restrict__ grad_out) {
    __shared__ double As[kXK][kXT + 1];
    __shared__ double Bs[kXK][kXT + 1];
    __shared__ double red[16][kXT + 1];
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const int64_t g0 = (int64_t)blockIdx.x * kXT;
    const int64_t plane = (int64_t)N * G;
    double part[4][4] = {};
    for (int nu0 = 0; nu0 < N; nu0 += kXT) {
        double acc[4][4] = {};
        for (int k0 = 0; k0 < N; k0 += kXK) {
            for (int t = threadIdx.x; t < kXK * kXT; t += 256) {
                const int kk = t % kXK, mm = t / kXK;
                const int r = nu0 + mm, k = k0 + kk;
                As[kk][mm] = (r < N && k < N) ? D[(int64_t)r * N + k] : 0.0;
            }
            for (int t = threadIdx.x; t < kXK * kXT; t += 256) {
                const int kk = t / kXT, nn = t % kXT;
                const int k = k0 + kk;
                Bs[kk][nn] = k < N ? phiT[(int64_t)k * G + g0 + nn] : 0.0;
            }
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < kXK; ++kk) {
                double a[4], b[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
                for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx + 16 * j];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
            }
            __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int nu = nu0 + ty + 16 * i;
            if (nu >= N) continue;
            const int64_t o = (int64_t)nu * G + g0 + tx;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                part[0][j] = fma(phiT[o + 16 * j], acc[i][j], part[0][j]);
#pragma unroll
                for (int k = 0; k < 3; ++k) part[1 + k][j] = fma(dphiT[k * plane + o + 16 * j], acc[i][j], part[1 + k][j]);
            }
        }
    }
    // fixed-order reductions over the 16 row groups, one quantity at a time
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int j = 0; j < 4; ++j) red[ty][tx + 16 * j] = part[q][j];
        __syncthreads();
        if (threadIdx.x < kXT) {
            double r = 0.0;
            for (int k = 0; k < 16; ++k) r += red[k][threadIdx.x];
            const int64_t g = g0 + threadIdx.x;
            if (q == 0) rho_out[g] = r;
            else grad_out[(q - 1) * G + g] = 2.0 * r;
        }
        __syncthreads();
    }
}

// The functional per point: energy partial sums per 256-point block (fixed
// order), f_g = w f_rho / 2 and hv[k][g] = 2 w f_sigma d_k rho.
__global__ void __launch_bounds__(256) k_pbe_point(int64_t G, const double *__restrict__ xyzw,
                                                   const double *__restrict__ rho, const double *__restrict__ grad,
                                                   double *__restrict__ f, double *__restrict__ hv,
                                                   double *__restrict__ epart) {
    __shared__ double red[256];
    const int64_t g = blockIdx.x * (int64_t)256 + threadIdx.x;
    double e = 0.0;
    if (g < G) {
        const double w = xyzw[4 * g + 3];
        const double gx = grad[g], gy = grad[G + g], gz = grad[2 * G + g];
        double fv, fr, fs;
        pbe_point(rho[g], gx * gx + gy * gy + gz * gz, fv, fr, fs);
        e = w * fv;
        f[g] = 0.5 * w * fr;
        const double h = 2.0 * w * fs;
        hv[g] = h * gx;
        hv[G + g] = h * gy;
        hv[2 * G + g] = h * gz;
    }
    red[threadIdx.x] = e;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) epart[blockIdx.x] = red[0];
}

// Vacc[mu][nu] += sum_{g in chunk} PhiT[mu][g] Z[nu][g] for every tile pair
// (bi, bj) = blockIdx.y, with Z[nu][g] = f_g PhiT[nu][g] + hv[.][g] . dPhiT[.][nu][g]
// formed as the tile is staged; V = Vacc + Vacc^T afterwards.
__global__ void __launch_bounds__(256) k_gga_v(int N, int64_t G, int nblk, const double *__restrict__ phiT,
                                               const double *__restrict__ dphiT, const double *__restrict__ f,
                                               const double *__restrict__ hv, double *__restrict__ Vacc) {
    __shared__ double As[kXK][kXT + 1];
    __shared__ double Bs[kXK][kXT + 1];
    const int bi = blockIdx.y / nblk, bj = blockIdx.y % nblk;
    const int row0 = bi * kXT, col0 = bj * kXT;
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const int64_t plane = (int64_t)N * G;
    const int64_t gs = (int64_t)blockIdx.x * kVChunk;
    const int64_t ge = gs + kVChunk < G ? gs + kVChunk : G;
    double acc[4][4] = {};
    for (int64_t k0 = gs; k0 < ge; k0 += kXK) {
        for (int t = threadIdx.x; t < kXK * kXT; t += 256) {
            const int kk = t % kXK, mm = t / kXK;
            const int r = row0 + mm;
            As[kk][mm] = r < N ? phiT[(int64_t)r * G + k0 + kk] : 0.0;
        }
        for (int t = threadIdx.x; t < kXK * kXT; t += 256) {
            const int kk = t % kXK, nn = t / kXK;
            const int c = col0 + nn;
            const int64_t g = k0 + kk, o = (int64_t)c * G + g;
            Bs[kk][nn] = c < N ? f[g] * phiT[o] + hv[g] * dphiT[o] + hv[G + g] * dphiT[plane + o] +
                                     hv[2 * G + g] * dphiT[2 * plane + o]
                               : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kXK; ++kk) {
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx + 16 * j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = row0 + ty + 16 * i;
        if (r >= N) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int c = col0 + tx + 16 * j;
            if (c < N) unsafeAtomicAdd(&Vacc[(int64_t)r * N + c], acc[i][j]);
        }
    }
}

// V = Vacc + Vacc^T (exactly symmetric)
__global__ void k_gga_sym(int N, const double *__restrict__ Vacc, double *__restrict__ V) {
    const int64_t NN = (int64_t)N * N;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < NN; idx += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(idx / N), j = (int)(idx % N);
        V[idx] = Vacc[idx] + Vacc[(int64_t)j * N + i];
    }
}

int zero_async(double *p, int64_t n, hipStream_t s);

// Grid and basis values, built once per basis (synchronous).
static int get_xc(mess_basis *B, XcGrid **out) {
    if (B->xc) {
        *out = static_cast<XcGrid *>(B->xc);
        return MESS_OK;
    }
    if (B->n_mol != 1) {
        set_error("LDA exchange is built for a single molecule, not a batch of %d", B->n_mol);
        return MESS_E_UNSUPPORTED;
    }
    auto *X = new XcGrid();
    B->xc = X;
    X->npts = (int64_t)B->nat * kPtsPerAtom;
    X->G = (X->npts + kXT - 1) / kXT * kXT;
    X->nbf = B->nbf;
    X->nrho_blocks = (int)(X->G / kXT);
    // radial (r, w) and angular (ux, uy, uz, w) rules
    std::vector<double> rad(2 * kNRad), ang(4 * kNAng);
    for (int i = 1; i <= kNRad; ++i) {
        const double t = i * M_PI / (kNRad + 1), x = std::cos(t);
        const double r = (1.0 + x) / (1.0 - x);
        rad[2 * (i - 1)] = r;
        rad[2 * (i - 1) + 1] = M_PI / (kNRad + 1) * std::sin(t) * 2.0 / ((1.0 - x) * (1.0 - x)) * r * r;
    }
    std::vector<double> u, a;
    gauss_legendre(kNTheta, u, a);
    for (int j = 0; j < kNTheta; ++j)
        for (int k = 0; k < kNPhi; ++k) {
            const double ph = 2.0 * M_PI * k / kNPhi, st = std::sqrt(1.0 - u[j] * u[j]);
            double *d = &ang[4 * (j * kNPhi + k)];
            d[0] = st * std::cos(ph);
            d[1] = st * std::sin(ph);
            d[2] = u[j];
            d[3] = a[j] * (2.0 * M_PI / kNPhi);
        }
    std::vector<XcShell> hs(B->nsh);
    for (int s = 0; s < B->nsh; ++s) {
        const int at = B->sh_atom[s];
        hs[s] = XcShell{B->xyz[3 * at], B->xyz[3 * at + 1], B->xyz[3 * at + 2], B->sh_l[s], B->sh_prim0[s],
                        B->sh_np[s], B->sh_bf0[s]};
    }
    double *d_rad = nullptr, *d_ang = nullptr, *d_alpha = nullptr, *d_ct = nullptr;
    XcShell *d_sh = nullptr;
    auto cleanup = [&]() {
        hipFree(d_rad);
        hipFree(d_ang);
        hipFree(d_alpha);
        hipFree(d_ct);
        hipFree(d_sh);
    };
    const size_t np = B->alpha.size();
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t r) {
        if (e == hipSuccess) e = r;
    };
    chk(hipMalloc(&X->xyzw, sizeof(double) * 4 * X->G));
    chk(hipMalloc(&X->phiT, sizeof(double) * (size_t)X->nbf * X->G));
    chk(hipMalloc(&X->f, sizeof(double) * X->G));
    chk(hipMalloc(&X->rho, sizeof(double) * X->G));
    chk(hipMalloc(&X->epart, sizeof(double) * X->nrho_blocks));
    chk(hipMalloc(&X->ex, sizeof(double)));
    chk(hipMalloc(&X->Vacc, sizeof(double) * (size_t)X->nbf * X->nbf));
    chk(hipMalloc(&d_rad, sizeof(double) * rad.size()));
    chk(hipMalloc(&d_ang, sizeof(double) * ang.size()));
    chk(hipMalloc(&d_alpha, sizeof(double) * np));
    chk(hipMalloc(&d_ct, sizeof(double) * np));
    chk(hipMalloc(&d_sh, sizeof(XcShell) * B->nsh));
    if (e != hipSuccess) {
        cleanup();
        free_xc(B);
        set_error("LDA grid: device allocation failed (%s)", hipGetErrorString(e));
        return MESS_E_NOMEM;
    }
    chk(hipMemcpy(d_rad, rad.data(), sizeof(double) * rad.size(), hipMemcpyHostToDevice));
    chk(hipMemcpy(d_ang, ang.data(), sizeof(double) * ang.size(), hipMemcpyHostToDevice));
    chk(hipMemcpy(d_alpha, B->alpha.data(), sizeof(double) * np, hipMemcpyHostToDevice));
    chk(hipMemcpy(d_ct, B->ctilde.data(), sizeof(double) * np, hipMemcpyHostToDevice));
    chk(hipMemcpy(d_sh, hs.data(), sizeof(XcShell) * B->nsh, hipMemcpyHostToDevice));
    if (e == hipSuccess) {
        const unsigned nb = (unsigned)((X->G + 255) / 256);
        hipLaunchKernelGGL(k_grid, dim3(nb), dim3(256), 0, nullptr, B->nat, B->d_xyz, d_rad, d_ang, X->npts, X->G,
                           X->xyzw);
        hipLaunchKernelGGL(k_basis_values, dim3(nb), dim3(256), 0, nullptr, B->nsh, d_sh, d_alpha, d_ct, X->npts,
                           X->G, X->xyzw, X->phiT);
        chk(hipGetLastError());
        chk(hipDeviceSynchronize());
    }
    cleanup();
    if (e != hipSuccess) {
        free_xc(B);
        set_error("LDA grid construction failed: %s", hipGetErrorString(e));
        return MESS_E_DEVICE;
    }
    *out = X;
    return MESS_OK;
}

// Basis gradients on the grid and the PBE per-point buffers, built on the
// first PBE call (synchronous).
static int ensure_gga(mess_basis *B, XcGrid *X) {
    if (X->dphiT) return MESS_OK;
    std::vector<XcShell> hs(B->nsh);
    for (int s = 0; s < B->nsh; ++s) {
        const int at = B->sh_atom[s];
        hs[s] = XcShell{B->xyz[3 * at], B->xyz[3 * at + 1], B->xyz[3 * at + 2], B->sh_l[s], B->sh_prim0[s],
                        B->sh_np[s], B->sh_bf0[s]};
    }
    const size_t np = B->alpha.size();
    double *d_alpha = nullptr, *d_ct = nullptr;
    XcShell *d_sh = nullptr;
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t r) {
        if (e == hipSuccess) e = r;
    };
    chk(hipMalloc(&X->dphiT, sizeof(double) * 3 * (size_t)X->nbf * X->G));
    chk(hipMalloc(&X->grad, sizeof(double) * 3 * X->G));
    chk(hipMalloc(&X->hv, sizeof(double) * 3 * X->G));
    chk(hipMalloc(&d_alpha, sizeof(double) * np));
    chk(hipMalloc(&d_ct, sizeof(double) * np));
    chk(hipMalloc(&d_sh, sizeof(XcShell) * B->nsh));
    if (e == hipSuccess) {
        chk(hipMemcpy(d_alpha, B->alpha.data(), sizeof(double) * np, hipMemcpyHostToDevice));
        chk(hipMemcpy(d_ct, B->ctilde.data(), sizeof(double) * np, hipMemcpyHostToDevice));
        chk(hipMemcpy(d_sh, hs.data(), sizeof(XcShell) * B->nsh, hipMemcpyHostToDevice));
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_basis_grad, dim3((unsigned)((X->G + 255) / 256)), dim3(256), 0, nullptr, B->nsh, d_sh,
                           d_alpha, d_ct, X->npts, X->G, X->nbf, X->xyzw, X->dphiT);
        chk(hipGetLastError());
        chk(hipDeviceSynchronize());
    }
    hipFree(d_alpha);
    hipFree(d_ct);
    hipFree(d_sh);
    if (e != hipSuccess) {
        for (double **p : {&X->dphiT, &X->grad, &X->hv}) {
            hipFree(*p);
            *p = nullptr;
        }
        set_error("PBE basis gradients: %s", hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? MESS_E_NOMEM : MESS_E_DEVICE;
    }
    return MESS_OK;
}

// PBE: V (device N x N, may be NULL) and the device scalar X->ex (E_xc)
// from density D.
int pbe_xc_async(mess_basis *B, const double *D, double *V, hipStream_t s, const double **ex_dev) {
    XcGrid *X = nullptr;
    MESS_TRY(get_xc(B, &X));
    MESS_TRY(ensure_gga(B, X));
    const int N = X->nbf;
    const unsigned npb = (unsigned)((X->G + 255) / 256);
    hipLaunchKernelGGL(k_gga_rho, dim3((unsigned)X->nrho_blocks), dim3(256), 0, s, N, X->G, D, X->phiT, X->dphiT,
                       X->rho, X->grad);
    hipLaunchKernelGGL(k_pbe_point, dim3(npb), dim3(256), 0, s, X->G, X->xyzw, X->rho, X->grad, X->f, X->hv,
                       X->epart);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, (int)npb, X->epart, X->ex);
    MESS_LAUNCH_CHECK();
    if (V) {
        const int nblk = (N + kXT - 1) / kXT;
        const unsigned chunks = (unsigned)((X->G + kVChunk - 1) / kVChunk);
        MESS_TRY(zero_async(X->Vacc, (int64_t)N * N, s));
        hipLaunchKernelGGL(k_gga_v, dim3(chunks, nblk * nblk), dim3(256), 0, s, N, X->G, nblk, X->phiT, X->dphiT,
                           X->f, X->hv, X->Vacc);
        hipLaunchKernelGGL(k_gga_sym, dim3(256), dim3(256), 0, s, N, X->Vacc, V);
        MESS_LAUNCH_CHECK();
    }
    if (ex_dev) *ex_dev = X->ex;
    return MESS_OK;
}

// V (device N x N, may be NULL) and the device scalar X->ex from density D.
int lda_x_async(mess_basis *B, const double *D, double *V, hipStream_t s, const double **ex_dev) {
    XcGrid *X = nullptr;
    MESS_TRY(get_xc(B, &X));
    const int N = X->nbf;
    hipLaunchKernelGGL(k_lda_rho, dim3((unsigned)X->nrho_blocks), dim3(256), 0, s, N, X->G, D, X->phiT, X->xyzw,
                       X->rho, X->f, X->epart);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, X->nrho_blocks, X->epart, X->ex);
    MESS_LAUNCH_CHECK();
    if (V) {
        const int nblk = (N + kXT - 1) / kXT;
        const unsigned chunks = (unsigned)((X->G + kVChunk - 1) / kVChunk);
        MESS_TRY(zero_async(X->Vacc, (int64_t)N * N, s));
        hipLaunchKernelGGL(k_lda_v, dim3(chunks, nblk * (nblk + 1) / 2), dim3(256), 0, s, N, X->G, nblk, X->phiT,
                           X->f, X->Vacc);
        hipLaunchKernelGGL(k_lda_mirror, dim3(256), dim3(256), 0, s, N, X->Vacc, V);
        MESS_LAUNCH_CHECK();
    }
    if (ex_dev) *ex_dev = X->ex;
    return MESS_OK;
}

int64_t lda_points(const mess_basis *B) { return (int64_t)B->nat * kPtsPerAtom; }

}  // namespace mess

using namespace mess;

extern "C" {

int mess_lda_x(const mess_basis *basis, const double *D, double *Vx, double *Ex, double *rho, mess_stream stream) {
    if (!basis || !D) {
        set_error("mess_lda_x: NULL basis or density");
        return MESS_E_ARG;
    }
    auto *B = const_cast<mess_basis *>(basis);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const double *ex = nullptr;
    MESS_TRY(lda_x_async(B, D, Vx, s, &ex));
    XcGrid *X = static_cast<XcGrid *>(B->xc);
    if (rho) MESS_HIP(hipMemcpyAsync(rho, X->rho, sizeof(double) * X->npts, hipMemcpyDeviceToDevice, s));
    if (Ex) {
        MESS_HIP(hipMemcpyAsync(Ex, ex, sizeof(double), hipMemcpyDeviceToHost, s));
        MESS_HIP(hipStreamSynchronize(s));
    }
    return MESS_OK;
}

int mess_pbe_xc(const mess_basis *basis, const double *D, double *Vxc, double *Exc, double *rho, double *grad_rho,
                mess_stream stream) {
    if (!basis || !D) {
        set_error("mess_pbe_xc: NULL basis or density");
        return MESS_E_ARG;
    }
    auto *B = const_cast<mess_basis *>(basis);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const double *ex = nullptr;
    MESS_TRY(pbe_xc_async(B, D, Vxc, s, &ex));
    XcGrid *X = static_cast<XcGrid *>(B->xc);
    if (rho) MESS_HIP(hipMemcpyAsync(rho, X->rho, sizeof(double) * X->npts, hipMemcpyDeviceToDevice, s));
    if (grad_rho)
        for (int k = 0; k < 3; ++k)
            MESS_HIP(hipMemcpyAsync(grad_rho + k * X->npts, X->grad + k * X->G, sizeof(double) * X->npts,
                                    hipMemcpyDeviceToDevice, s));
    if (Exc) {
        MESS_HIP(hipMemcpyAsync(Exc, ex, sizeof(double), hipMemcpyDeviceToHost, s));
        MESS_HIP(hipStreamSynchronize(s));
    }
    return MESS_OK;
}

int mess_grid(const mess_basis *basis, double *xyzw, int64_t *npts, mess_stream stream) {
    if (!basis) {
        set_error("mess_grid: NULL basis");
        return MESS_E_ARG;
    }
    auto *B = const_cast<mess_basis *>(basis);
    if (B->n_mol != 1) {
        set_error("mess_grid: LDA grids are built for a single molecule, not a batch of %d", B->n_mol);
        return MESS_E_UNSUPPORTED;
    }
    if (npts) *npts = lda_points(B);
    if (!xyzw) return MESS_OK;
    XcGrid *X = nullptr;
    MESS_TRY(get_xc(B, &X));
    MESS_HIP(hipMemcpyAsync(xyzw, X->xyzw, sizeof(double) * 4 * X->npts, hipMemcpyDeviceToDevice,
                            static_cast<hipStream_t>(stream)));
    return MESS_OK;
}

}  // extern "C"
