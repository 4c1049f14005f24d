// Learned initial density guess: atom-pair features, a 64 -> 256 -> 256 ->
// 128 perceptron (SiLU hidden layers) whose outputs are density blocks,
// assembly into a packed block-diagonal density, and training by masked
// mean-squared error with Adam.  Every layer product runs on the BF16
// matrix cores (v_mfma_f32_16x16x16_bf16): operands are rounded to BF16
// (nearest, ties to even), products accumulate in FP32, and biases,
// pre-activations, gradients and the Adam state stay FP32.
//
// Pair rows: for each molecule, atoms A <= B in A-major order.  Features
// (42 of 64 used): one-hot element of A and B over (H, C, N, O); 16
// Gaussian radial functions of R_AB (centres k 10/15, width 10/15 bohr);
// the unit vector A -> B and its six products; per-element neighbour counts
// of A and B with the cutoff (cos(pi R/6) + 1)/2 below 6 bohr; a self-pair
// flag.  Output 11 i + j is the density element between function i of A and
// function j of B.
#include <algorithm>
#include <cmath>
#include <vector>

#include "mess_internal.hpp"

namespace mess {

constexpr int kIn = 64, kHid = 256, kOut = 128, kBlk = 11;
constexpr int64_t kOffW1 = 0, kOffB1 = kOffW1 + kHid * kIn, kOffW2 = kOffB1 + kHid,
                  kOffB2 = kOffW2 + kHid * kHid, kOffW3 = kOffB2 + kHid, kOffB3 = kOffW3 + kOut * kHid,
                  kNParam = kOffB3 + kOut;
static_assert(kNParam == MESS_MLP_NPARAM, "parameter layout");

struct PairRow {
    int64_t moff;    // packed block of the molecule
    int n;           // functions of the molecule
    int fa, na;      // first function (within the molecule) and count of atom A
    int fb, nb;      // same for atom B
    int self, pad;
};

struct GuessTables {
    int64_t nrows = 0;
    std::vector<PairRow> rows;
    std::vector<float> feat;   // [nrows][64]
    PairRow *d_rows = nullptr;
};

void free_guess_tables(mess_basis *B) {
    auto *T = static_cast<GuessTables *>(B->guess);
    if (!T) return;
    hipFree(T->d_rows);
    delete T;
    B->guess = nullptr;
}

static int element_index(int Z) { return Z == 1 ? 0 : Z == 6 ? 1 : Z == 7 ? 2 : Z == 8 ? 3 : -1; }

static int get_tables(mess_basis *B, GuessTables **out) {
    if (B->guess) {
        *out = static_cast<GuessTables *>(B->guess);
        return MESS_OK;
    }
    auto *T = new GuessTables();
    for (int m = 0; m < B->n_mol; ++m) {
        const int a0 = B->mol_atom0[m], na = B->mol_natom[m];
        std::vector<int> first(na, -1), count(na, 0), el(na);
        int last = -1;
        for (int s = B->mol_sh0[m]; s < B->mol_sh0[m] + B->mol_nsh[m]; ++s) {
            const int a = B->sh_atom[s] - a0;
            if (first[a] < 0) {
                if (a < last) goto noncontig;
                first[a] = B->sh_bf0[s] - B->mol_bf0[m];
            } else if (a != last) {
                goto noncontig;
            }
            last = a;
            count[a] += ncart(B->sh_l[s]);
        }
        for (int a = 0; a < na; ++a) {
            el[a] = element_index(B->Z[a0 + a]);
            if (el[a] < 0 || count[a] == 0 || count[a] > kBlk) {
                delete T;
                set_error("learned guess: atom %d of molecule %d has Z=%d and %d functions (H, C, N, O with 1..11 "
                          "functions are supported)",
                          a, m, B->Z[a0 + a], count[a]);
                return MESS_E_UNSUPPORTED;
            }
        }
        {
            const double *X = &B->xyz[3 * a0];
            std::vector<double> cnt(4 * na, 0.0);
            for (int a = 0; a < na; ++a)
                for (int c = 0; c < na; ++c) {
                    if (c == a) continue;
                    const double dx = X[3 * a] - X[3 * c], dy = X[3 * a + 1] - X[3 * c + 1],
                                 dz = X[3 * a + 2] - X[3 * c + 2];
                    const double r = std::sqrt(dx * dx + dy * dy + dz * dz);
                    if (r < 6.0) cnt[4 * a + el[c]] += 0.5 * (std::cos(M_PI * r / 6.0) + 1.0);
                }
            for (int a = 0; a < na; ++a)
                for (int b = a; b < na; ++b) {
                    PairRow pr{B->mol_moff[m], B->mol_nbf[m], first[a], count[a], first[b], count[b], a == b, 0};
                    T->rows.push_back(pr);
                    double f[kIn] = {0.0};
                    f[el[a]] = 1.0;
                    f[4 + el[b]] = 1.0;
                    const double dx = X[3 * b] - X[3 * a], dy = X[3 * b + 1] - X[3 * a + 1],
                                 dz = X[3 * b + 2] - X[3 * a + 2];
                    const double r = std::sqrt(dx * dx + dy * dy + dz * dz);
                    const double sig = 10.0 / 15.0;
                    for (int k = 0; k < 16; ++k) {
                        const double t = (r - k * sig) / sig;
                        f[8 + k] = std::exp(-(t * t));
                    }
                    if (a != b) {
                        const double u[3] = {dx / r, dy / r, dz / r};
                        f[24] = u[0];
                        f[25] = u[1];
                        f[26] = u[2];
                        f[27] = u[0] * u[0];
                        f[28] = u[0] * u[1];
                        f[29] = u[0] * u[2];
                        f[30] = u[1] * u[1];
                        f[31] = u[1] * u[2];
                        f[32] = u[2] * u[2];
                    }
                    for (int e = 0; e < 4; ++e) {
                        f[33 + e] = cnt[4 * a + e];
                        f[37 + e] = cnt[4 * b + e];
                    }
                    f[41] = a == b ? 1.0 : 0.0;
                    for (int k = 0; k < kIn; ++k) T->feat.push_back((float)f[k]);
                }
        }
        continue;
    noncontig:
        delete T;
        set_error("learned guess: the shells of an atom of molecule %d are not contiguous", m);
        return MESS_E_UNSUPPORTED;
    }
    T->nrows = (int64_t)T->rows.size();
    if (hipMalloc(&T->d_rows, sizeof(PairRow) * std::max<int64_t>(T->nrows, 1)) != hipSuccess ||
        hipMemcpy(T->d_rows, T->rows.data(), sizeof(PairRow) * T->nrows, hipMemcpyHostToDevice) != hipSuccess) {
        hipFree(T->d_rows);
        delete T;
        set_error("learned guess: cannot allocate pair tables");
        return MESS_E_NOMEM;
    }
    B->guess = T;
    *out = T;
    return MESS_OK;
}

// T[r][11 i + j] = D block element, M = 1 inside the block (0 elsewhere).
__global__ void k_guess_targets(int64_t nrows, const PairRow *__restrict__ rows, const double *__restrict__ D,
                                float *__restrict__ T, float *__restrict__ M) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= nrows * kOut) return;
    const int64_t r = t / kOut;
    const int k = (int)(t % kOut), i = k / kBlk, j = k % kBlk;
    const PairRow p = rows[r];
    const bool in = k < kBlk * kBlk && i < p.na && j < p.nb;
    if (T) T[t] = in ? (float)D[p.moff + (int64_t)(p.fa + i) * p.n + p.fb + j] : 0.0f;
    if (M) M[t] = in ? 1.0f : 0.0f;
}

// D[A_i][B_j] = D[B_j][A_i] = Y[r][11 i + j]; diagonal blocks symmetrised.
__global__ void k_guess_assemble(int64_t nrows, const PairRow *__restrict__ rows, const float *__restrict__ Y,
                                 double *__restrict__ D) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= nrows * kBlk * kBlk) return;
    const int64_t r = t / (kBlk * kBlk);
    const int k = (int)(t % (kBlk * kBlk)), i = k / kBlk, j = k % kBlk;
    const PairRow p = rows[r];
    if (i >= p.na || j >= p.nb) return;
    const float *y = Y + r * kOut;
    const double v = p.self ? 0.5 * ((double)y[kBlk * i + j] + (double)y[kBlk * j + i]) : (double)y[kBlk * i + j];
    D[p.moff + (int64_t)(p.fa + i) * p.n + p.fb + j] = v;
    D[p.moff + (int64_t)(p.fb + j) * p.n + p.fa + i] = v;
}

// ------------------------------------------------------------ BF16 MFMA

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short to_bf16(float x) {
    unsigned u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

__device__ __forceinline__ float silu_f(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float dsilu_f(float z) {
    const float s = 1.0f / (1.0f + expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

enum { kEpiHidden = 0, kEpiOut = 1, kEpiBackHidden = 2, kEpiAtomic = 3 };

constexpr int kGT = 64;   // output tile edge
constexpr int kGK = 32;   // K per LDS stage (two MFMA steps)
constexpr int kLdsK = kGK + 4;  // row stride (bf16 elements), 8-byte aligned fragments

// C[M x N] = op(A)[M x K] op(B)[K x N] with BF16 operands and FP32
// accumulation.  op(A) = A (M x K row-major, lda) or, with TA, A stored
// K x M; op(B) = B (K x N row-major) or, with TB, B stored N x K.
// Epilogues:
//   kEpiHidden:     Zf = acc + bias[n];  Hb = bf16(silu(Zf))
//   kEpiOut:        Zf = acc + bias[n]
//   kEpiBackHidden: Zf = acc * dsilu(aux[m][n]);  Hb = bf16(Zf)
//   kEpiAtomic:     Zf[m][n] += acc (split K over blockIdx.z, kSplit rows each)
// A 256-thread block computes a 64 x 64 tile; wave w owns the 32 x 32
// quadrant (w / 2, w % 2) as 2 x 2 MFMA 16 x 16 tiles.  MFMA operand
// layout (16 x 16 x 16): lane l holds A[l % 16][4 (l / 16) + 0..3],
// B[4 (l / 16) + 0..3][l % 16], and the result rows 4 (l / 16) + 0..3 of
// column l % 16.
template <bool TA, bool TB, int EPI>
__global__ void __launch_bounds__(256) k_gemm_bf16(int M, int N, int K, int kSplit,
                                                   const unsigned short *__restrict__ A, int lda,
                                                   const unsigned short *__restrict__ B, int ldb,
                                                   const float *__restrict__ bias, const float *__restrict__ aux,
                                                   float *__restrict__ Zf, unsigned short *__restrict__ Hb, int ldc) {
    __shared__ __align__(16) unsigned short As[kGT][kLdsK];
    __shared__ __align__(16) unsigned short Bs[kGT][kLdsK];  // [n][k]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m0 = blockIdx.y * kGT, n0 = blockIdx.x * kGT;
    const int kbeg = EPI == kEpiAtomic ? blockIdx.z * kSplit : 0;
    const int kend = EPI == kEpiAtomic ? min(K, kbeg + kSplit) : K;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    v4f acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = kbeg; k0 < kend; k0 += kGK) {
        // stage A tile [64 m][32 k] and B tile [64 n][32 k]
        for (int t = threadIdx.x; t < kGT * kGK; t += 256) {
            int m, k;
            if (TA) {
                k = t / kGT;
                m = t % kGT;  // global contiguous in m
            } else {
                m = t / kGK;
                k = t % kGK;  // contiguous in k
            }
            const int gm = m0 + m, gk = k0 + k;
            unsigned short v = 0;
            if (gm < M && gk < kend) v = TA ? A[(int64_t)gk * lda + gm] : A[(int64_t)gm * lda + gk];
            As[m][k] = v;
        }
        for (int t = threadIdx.x; t < kGT * kGK; t += 256) {
            int n, k;
            if (TB) {
                n = t / kGK;
                k = t % kGK;
            } else {
                k = t / kGT;
                n = t % kGT;
            }
            const int gn = n0 + n, gk = k0 + k;
            unsigned short v = 0;
            if (gn < N && gk < kend) v = TB ? B[(int64_t)gn * ldb + gk] : B[(int64_t)gk * ldb + gn];
            Bs[n][k] = v;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kGK; ks += 16) {
            const int kk = ks + 4 * (lane >> 4);
            v4s a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = *reinterpret_cast<const v4s *>(&As[wm + 16 * i + (lane & 15)][kk]);
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = *reinterpret_cast<const v4s *>(&Bs[wn + 16 * j + (lane & 15)][kk]);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gm = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
                const int gn = n0 + wn + 16 * j + (lane & 15);
                if (gm >= M || gn >= N) continue;
                const int64_t o = (int64_t)gm * ldc + gn;
                const float v = acc[i][j][r];
                if (EPI == kEpiHidden) {
                    const float z = v + bias[gn];
                    Zf[o] = z;
                    Hb[o] = to_bf16(silu_f(z));
                } else if (EPI == kEpiOut) {
                    Zf[o] = v + bias[gn];
                } else if (EPI == kEpiBackHidden) {
                    const float z = v * dsilu_f(aux[o]);
                    Zf[o] = z;
                    Hb[o] = to_bf16(z);
                } else {
                    unsafeAtomicAdd(&Zf[o], v);
                }
            }
}

__global__ void k_to_bf16(int64_t n, const float *__restrict__ x, unsigned short *__restrict__ y) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = to_bf16(x[i]);
}

__global__ void k_fill_f32(int64_t n, float *__restrict__ p) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

// sum of the mask (one block)
__global__ void __launch_bounds__(256) k_mask_sum(int64_t n, const float *__restrict__ M, float *__restrict__ out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) s += M[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = (float)red[0];
}

// dY = 2 M (Y - T) / sum(M) (FP32 and BF16); per-block partial sums of
// M (Y - T)^2 (FP64).
__global__ void __launch_bounds__(256) k_mse(int64_t n, const float *__restrict__ Y, const float *__restrict__ T,
                                             const float *__restrict__ M, const float *__restrict__ msum,
                                             float *__restrict__ dY, unsigned short *__restrict__ dYb,
                                             double *__restrict__ part) {
    __shared__ double red[256];
    const float inv = 2.0f / msum[0];
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float d = M[i] * (Y[i] - T[i]);
        s += (double)d * d;
        const float g = d * inv;
        dY[i] = g;
        dYb[i] = to_bf16(g);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) k_loss_finish(int nb, const double *__restrict__ part,
                                                     const float *__restrict__ msum, double *__restrict__ loss) {
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = red[0] / (double)msum[0];
}

// db[j] = sum over rows of G[r][j] (FP32), one thread per column, rows split
// over blockIdx.y with atomics.
__global__ void k_colsum(int64_t nrows, int ncol, int rows_per, const float *__restrict__ G, float *__restrict__ db) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ncol) return;
    const int64_t r0 = (int64_t)blockIdx.y * rows_per;
    const int64_t r1 = r0 + rows_per < nrows ? r0 + rows_per : nrows;
    float s = 0.0f;
    for (int64_t r = r0; r < r1; ++r) s += G[r * ncol + j];
    unsafeAtomicAdd(&db[j], s);
}

__global__ void k_adam(int64_t n, float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, float lr, float b1, float b2, float eps, float c1, float c2,
                       unsigned short *__restrict__ pb) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        p[i] = pi;
        pb[i] = to_bf16(pi);
    }
}

}  // namespace mess

// ------------------------------------------------------------ the model

struct mess_mlp {
    float *p = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
    unsigned short *pb = nullptr;
    int t = 0;
    int64_t cap = 0;  // rows the workspace holds
    unsigned short *Xb = nullptr, *H1b = nullptr, *H2b = nullptr, *dYb = nullptr, *dZ2b = nullptr, *dZ1b = nullptr;
    float *Z1 = nullptr, *Z2 = nullptr, *dY = nullptr, *dZ2 = nullptr, *dZ1 = nullptr, *Yw = nullptr;
    float *msum = nullptr;
    double *part = nullptr, *loss = nullptr;
};

namespace mess {

constexpr int kMseBlocks = 512;

static void free_ws(mess_mlp *L) {
    for (void *q : {(void *)L->Xb, (void *)L->H1b, (void *)L->H2b, (void *)L->dYb, (void *)L->dZ2b, (void *)L->dZ1b,
                    (void *)L->Z1, (void *)L->Z2, (void *)L->dY, (void *)L->dZ2, (void *)L->dZ1, (void *)L->Yw})
        hipFree(q);
    L->Xb = L->H1b = L->H2b = L->dYb = L->dZ2b = L->dZ1b = nullptr;
    L->Z1 = L->Z2 = L->dY = L->dZ2 = L->dZ1 = L->Yw = nullptr;
    L->cap = 0;
}

static int ensure_ws(mess_mlp *L, int64_t n) {
    if (n <= L->cap) return MESS_OK;
    MESS_HIP(hipDeviceSynchronize());
    free_ws(L);
    hipError_t e = hipSuccess;
    auto al = [&](void **q, size_t bytes) {
        if (e == hipSuccess) e = hipMalloc(q, bytes);
    };
    al((void **)&L->Xb, 2 * n * kIn);
    al((void **)&L->H1b, 2 * n * kHid);
    al((void **)&L->H2b, 2 * n * kHid);
    al((void **)&L->dYb, 2 * n * kOut);
    al((void **)&L->dZ2b, 2 * n * kHid);
    al((void **)&L->dZ1b, 2 * n * kHid);
    al((void **)&L->Z1, 4 * n * kHid);
    al((void **)&L->Z2, 4 * n * kHid);
    al((void **)&L->dY, 4 * n * kOut);
    al((void **)&L->dZ2, 4 * n * kHid);
    al((void **)&L->dZ1, 4 * n * kHid);
    al((void **)&L->Yw, 4 * n * kOut);
    if (e != hipSuccess) {
        free_ws(L);
        set_error("perceptron workspace for %lld rows: %s", (long long)n, hipGetErrorString(e));
        return MESS_E_NOMEM;
    }
    L->cap = n;
    return MESS_OK;
}

static unsigned g1(int64_t n) { return (unsigned)std::min<int64_t>(std::max<int64_t>((n + 255) / 256, 1), 4096); }

template <bool TA, bool TB, int EPI>
static int gemm16(hipStream_t s, int M, int N, int K, const unsigned short *A, int lda, const unsigned short *Bm,
                  int ldb, const float *bias, const float *aux, float *Zf, unsigned short *Hb, int ldc) {
    int split = K, nz = 1;
    if (EPI == kEpiAtomic) {
        split = 1024;
        nz = (K + split - 1) / split;
    }
    dim3 grid((N + kGT - 1) / kGT, (M + kGT - 1) / kGT, nz);
    hipLaunchKernelGGL((k_gemm_bf16<TA, TB, EPI>), grid, dim3(256), 0, s, M, N, K, split, A, lda, Bm, ldb, bias, aux,
                       Zf, Hb, ldc);
    MESS_LAUNCH_CHECK();
    return MESS_OK;
}

// Forward over n rows of X (FP32): Y (FP32); keeps Z1, H1b, Z2, H2b.
static int mlp_forward(mess_mlp *L, int64_t n, const float *X, float *Y, hipStream_t s) {
    MESS_TRY(ensure_ws(L, n));
    const unsigned short *W1 = L->pb + kOffW1, *W2 = L->pb + kOffW2, *W3 = L->pb + kOffW3;
    hipLaunchKernelGGL(k_to_bf16, dim3(g1(n * kIn)), dim3(256), 0, s, n * kIn, X, L->Xb);
    MESS_LAUNCH_CHECK();
    const int nn = (int)n;
    MESS_TRY((gemm16<false, true, kEpiHidden>(s, nn, kHid, kIn, L->Xb, kIn, W1, kIn, L->p + kOffB1, nullptr, L->Z1,
                                              L->H1b, kHid)));
    MESS_TRY((gemm16<false, true, kEpiHidden>(s, nn, kHid, kHid, L->H1b, kHid, W2, kHid, L->p + kOffB2, nullptr,
                                              L->Z2, L->H2b, kHid)));
    MESS_TRY((gemm16<false, true, kEpiOut>(s, nn, kOut, kHid, L->H2b, kHid, W3, kHid, L->p + kOffB3, nullptr, Y,
                                           nullptr, kOut)));
    return MESS_OK;
}

// Loss and gradient (into L->g) of the masked MSE over n rows.
static int mlp_grad(mess_mlp *L, int64_t n, const float *X, const float *T, const float *M, hipStream_t s) {
    // the workspace (L->Yw among it) must exist before its pointers are taken
    MESS_TRY(ensure_ws(L, n));
    MESS_TRY(mlp_forward(L, n, X, L->Yw, s));
    const int nn = (int)n;
    const int64_t no = n * kOut;
    hipLaunchKernelGGL(k_mask_sum, dim3(1), dim3(256), 0, s, no, M, L->msum);
    hipLaunchKernelGGL(k_mse, dim3(kMseBlocks), dim3(256), 0, s, no, L->Yw, T, M, L->msum, L->dY, L->dYb, L->part);
    hipLaunchKernelGGL(k_loss_finish, dim3(1), dim3(256), 0, s, kMseBlocks, L->part, L->msum, L->loss);
    hipLaunchKernelGGL(k_fill_f32, dim3(g1(kNParam)), dim3(256), 0, s, (int64_t)kNParam, L->g);
    MESS_LAUNCH_CHECK();
    const unsigned short *W2 = L->pb + kOffW2, *W3 = L->pb + kOffW3;
    const int rows_per = 512;
    const unsigned ry = (unsigned)((n + rows_per - 1) / rows_per);
    // layer 3: dW3 = dY^T H2, db3 = sum dY, dZ2 = (dY W3) .* silu'(Z2)
    MESS_TRY((gemm16<true, false, kEpiAtomic>(s, kOut, kHid, nn, L->dYb, kOut, L->H2b, kHid, nullptr, nullptr,
                                              L->g + kOffW3, nullptr, kHid)));
    hipLaunchKernelGGL(k_colsum, dim3(1, ry), dim3(kOut), 0, s, n, kOut, rows_per, L->dY, L->g + kOffB3);
    MESS_TRY((gemm16<false, false, kEpiBackHidden>(s, nn, kHid, kOut, L->dYb, kOut, W3, kHid, nullptr, L->Z2, L->dZ2,
                                                   L->dZ2b, kHid)));
    // layer 2
    MESS_TRY((gemm16<true, false, kEpiAtomic>(s, kHid, kHid, nn, L->dZ2b, kHid, L->H1b, kHid, nullptr, nullptr,
                                              L->g + kOffW2, nullptr, kHid)));
    hipLaunchKernelGGL(k_colsum, dim3(1, ry), dim3(kHid), 0, s, n, kHid, rows_per, L->dZ2, L->g + kOffB2);
    MESS_TRY((gemm16<false, false, kEpiBackHidden>(s, nn, kHid, kHid, L->dZ2b, kHid, W2, kHid, nullptr, L->Z1,
                                                   L->dZ1, L->dZ1b, kHid)));
    // layer 1
    MESS_TRY((gemm16<true, false, kEpiAtomic>(s, kHid, kIn, nn, L->dZ1b, kHid, L->Xb, kIn, nullptr, nullptr,
                                              L->g + kOffW1, nullptr, kIn)));
    hipLaunchKernelGGL(k_colsum, dim3(1, ry), dim3(kHid), 0, s, n, kHid, rows_per, L->dZ1, L->g + kOffB1);
    MESS_LAUNCH_CHECK();
    return MESS_OK;
}

static void free_mlp(mess_mlp *L) {
    if (!L) return;
    free_ws(L);
    for (void *q : {(void *)L->p, (void *)L->m, (void *)L->v, (void *)L->g, (void *)L->pb, (void *)L->msum,
                    (void *)L->part, (void *)L->loss})
        hipFree(q);
    delete L;
}

static int check_rows(int64_t n, const char *who) {
    // grid.y = rows / 64 must stay below 65536
    if (n <= 0 || n > (int64_t)1 << 21) {
        set_error("%s: row count %lld out of range (1 .. 2^21)", who, (long long)n);
        return MESS_E_ARG;
    }
    return MESS_OK;
}

int guess_rows(mess_basis *B, int64_t *n) {
    GuessTables *T = nullptr;
    MESS_TRY(get_tables(B, &T));
    *n = T->nrows;
    return MESS_OK;
}

int guess_assemble_async(mess_basis *B, const float *Y, double *D, hipStream_t s) {
    GuessTables *T = nullptr;
    MESS_TRY(get_tables(B, &T));
    int zero_async(double *p, int64_t n, hipStream_t s);
    MESS_TRY(zero_async(D, B->packed, s));
    const int64_t nt = T->nrows * kBlk * kBlk;
    hipLaunchKernelGGL(k_guess_assemble, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, T->nrows, T->d_rows, Y,
                       D);
    MESS_LAUNCH_CHECK();
    return MESS_OK;
}

int guess_features_async(mess_basis *B, float *X, hipStream_t s) {
    GuessTables *T = nullptr;
    MESS_TRY(get_tables(B, &T));
    MESS_HIP(hipMemcpyAsync(X, T->feat.data(), sizeof(float) * T->feat.size(), hipMemcpyHostToDevice, s));
    MESS_HIP(hipStreamSynchronize(s));  // the host array is pageable
    return MESS_OK;
}

int mlp_forward_ext(mess_mlp *L, int64_t n, const float *X, float *Y, hipStream_t s) {
    return mlp_forward(L, n, X, Y, s);
}

}  // namespace mess

using namespace mess;

extern "C" {

int mess_mlp_create(const float *params, mess_mlp **out) {
    if (!params || !out) {
        set_error("mess_mlp_create: NULL parameters or output");
        return MESS_E_ARG;
    }
    *out = nullptr;
    auto *L = new mess_mlp();
    hipError_t e = hipSuccess;
    auto al = [&](void **q, size_t bytes) {
        if (e == hipSuccess) e = hipMalloc(q, bytes);
    };
    al((void **)&L->p, 4 * kNParam);
    al((void **)&L->m, 4 * kNParam);
    al((void **)&L->v, 4 * kNParam);
    al((void **)&L->g, 4 * kNParam);
    al((void **)&L->pb, 2 * kNParam);
    al((void **)&L->msum, 4);
    al((void **)&L->part, 8 * kMseBlocks);
    al((void **)&L->loss, 8);
    if (e == hipSuccess) e = hipMemcpy(L->p, params, 4 * kNParam, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(L->m, 0, 4 * kNParam);
    if (e == hipSuccess) e = hipMemset(L->v, 0, 4 * kNParam);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_to_bf16, dim3(g1(kNParam)), dim3(256), 0, nullptr, (int64_t)kNParam, L->p, L->pb);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        set_error("mess_mlp_create: %s", hipGetErrorString(e));
        free_mlp(L);
        return MESS_E_NOMEM;
    }
    *out = L;
    return MESS_OK;
}

void mess_mlp_destroy(mess_mlp *mlp) { free_mlp(mlp); }

int mess_mlp_params(const mess_mlp *mlp, float *params) {
    if (!mlp || !params) {
        set_error("mess_mlp_params: NULL argument");
        return MESS_E_ARG;
    }
    MESS_HIP(hipDeviceSynchronize());
    MESS_HIP(hipMemcpy(params, mlp->p, 4 * kNParam, hipMemcpyDeviceToHost));
    return MESS_OK;
}

int mess_mlp_forward(mess_mlp *mlp, int64_t n, const float *X, float *Y, mess_stream stream) {
    if (!mlp || !X || !Y) {
        set_error("mess_mlp_forward: NULL argument");
        return MESS_E_ARG;
    }
    MESS_TRY(check_rows(n, "mess_mlp_forward"));
    return mlp_forward(mlp, n, X, Y, static_cast<hipStream_t>(stream));
}

int mess_mlp_grad(mess_mlp *mlp, int64_t n, const float *X, const float *T, const float *M, float *grad,
                  double *loss, mess_stream stream) {
    if (!mlp || !X || !T || !M) {
        set_error("mess_mlp_grad: NULL argument");
        return MESS_E_ARG;
    }
    MESS_TRY(check_rows(n, "mess_mlp_grad"));
    hipStream_t s = static_cast<hipStream_t>(stream);
    MESS_TRY(mlp_grad(mlp, n, X, T, M, s));
    if (grad) MESS_HIP(hipMemcpyAsync(grad, mlp->g, 4 * kNParam, hipMemcpyDeviceToDevice, s));
    if (loss) {
        MESS_HIP(hipMemcpyAsync(loss, mlp->loss, 8, hipMemcpyDeviceToHost, s));
        MESS_HIP(hipStreamSynchronize(s));
    }
    return MESS_OK;
}

int mess_mlp_train_step(mess_mlp *mlp, int64_t n, const float *X, const float *T, const float *M, float lr,
                        double *loss, mess_stream stream) {
    if (!mlp || !X || !T || !M || !(lr > 0.0f)) {
        set_error("mess_mlp_train_step: NULL argument or learning rate <= 0");
        return MESS_E_ARG;
    }
    MESS_TRY(check_rows(n, "mess_mlp_train_step"));
    hipStream_t s = static_cast<hipStream_t>(stream);
    MESS_TRY(mlp_grad(mlp, n, X, T, M, s));
    mlp->t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - std::pow(b1, (float)mlp->t), c2 = 1.0f - std::pow(b2, (float)mlp->t);
    hipLaunchKernelGGL(k_adam, dim3(g1(kNParam)), dim3(256), 0, s, (int64_t)kNParam, mlp->p, mlp->m, mlp->v, mlp->g,
                       lr, b1, b2, 1e-8f, c1, c2, mlp->pb);
    MESS_LAUNCH_CHECK();
    if (loss) {
        MESS_HIP(hipMemcpyAsync(loss, mlp->loss, 8, hipMemcpyDeviceToHost, s));
        MESS_HIP(hipStreamSynchronize(s));
    }
    return MESS_OK;
}

int mess_guess_rows(const mess_basis *basis, int64_t *n_rows) {
    if (!basis || !n_rows) {
        set_error("mess_guess_rows: NULL argument");
        return MESS_E_ARG;
    }
    return guess_rows(const_cast<mess_basis *>(basis), n_rows);
}

int mess_guess_features(const mess_basis *basis, float *X, mess_stream stream) {
    if (!basis || !X) {
        set_error("mess_guess_features: NULL argument");
        return MESS_E_ARG;
    }
    return guess_features_async(const_cast<mess_basis *>(basis), X, static_cast<hipStream_t>(stream));
}

int mess_guess_targets(const mess_basis *basis, const double *D, float *T, float *M, mess_stream stream) {
    if (!basis || !D || (!T && !M)) {
        set_error("mess_guess_targets: NULL argument");
        return MESS_E_ARG;
    }
    GuessTables *G = nullptr;
    MESS_TRY(get_tables(const_cast<mess_basis *>(basis), &G));
    const int64_t nt = G->nrows * kOut;
    hipLaunchKernelGGL(k_guess_targets, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), G->nrows, G->d_rows, D, T, M);
    MESS_LAUNCH_CHECK();
    return MESS_OK;
}

int mess_guess_assemble(const mess_basis *basis, const float *Y, double *D, mess_stream stream) {
    if (!basis || !Y || !D) {
        set_error("mess_guess_assemble: NULL argument");
        return MESS_E_ARG;
    }
    return guess_assemble_async(const_cast<mess_basis *>(basis), Y, D, static_cast<hipStream_t>(stream));
}

}  // extern "C"
