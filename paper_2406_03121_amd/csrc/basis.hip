// Basis creation (normalisation, device tables), shell pairs, Schwarz
// factors and unique shell-quartet work lists.
#include <cmath>
#include <cstdarg>
#include <cstring>

#include "class_ops.hpp"
#include "mess_internal.hpp"

namespace mess {

// ------------------------------------------------------------- errors

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

// --------------------------------------------------------------- Boys
//
// Table of F_n(T_k), T_k = k/16, n < 16, built on the host in extended
// precision: F_15 from its power series
//   F_n(T) = e^{-T} sum_i (2T)^i / ((2n+1)(2n+3)...(2n+2i+1))
// (all terms positive), lower orders by the stable downward recurrence
//   F_n = (2T F_{n+1} + e^{-T}) / (2n+1).

static void build_boys_table(std::vector<double> &tab, std::vector<double> &etab) {
    tab.assign((size_t)kBoysRows * kBoysN, 0.0);
    etab.assign(kBoysRows, 0.0);
    for (int k = 0; k < kBoysRows; ++k) {
        const long double T = (long double)k / (long double)kBoysInvStep;
        const long double eT = expl(-T);
        const int n = kBoysN - 1;
        long double term = 1.0L / (2 * n + 1), sum = term;
        for (int i = 1; i < 4000; ++i) {
            term *= 2.0L * T / (long double)(2 * n + 2 * i + 1);
            sum += term;
            if (term < 1e-22L * sum) break;
        }
        long double F[kBoysN];
        F[n] = eT * sum;
        for (int m = n - 1; m >= 0; --m) F[m] = (2.0L * T * F[m + 1] + eT) / (long double)(2 * m + 1);
        for (int m = 0; m < kBoysN; ++m) tab[(size_t)k * kBoysN + m] = (double)F[m];
        etab[k] = (double)eT;
    }
}

// ------------------------------------------------ normalisation (host)
//
// Contracted shell of angular momentum l: phi = N_c sum_p c_p N(a_p; l,0,0) g_p
// with N(a; l,0,0) = (2a/pi)^{3/4} (4a)^{l/2} / sqrt((2l-1)!!) and
// N_c^{-2} = sum_pq c_p c_q (2 sqrt(a_p a_q)/(a_p+a_q))^{l+3/2}.
// The remaining per-component factor sqrt((2l-1)!!/((2lx-1)!!(2ly-1)!!(2lz-1)!!))
// is applied to integrals at output time.

static double dfact_odd(int n) {
    double r = 1.0;
    for (int k = n; k > 1; k -= 2) r *= k;
    return r;
}

static void normalise(const int l, const int np, const double *a, const double *c, double *out) {
    double s = 0.0;
    for (int p = 0; p < np; ++p)
        for (int q = 0; q < np; ++q)
            s += c[p] * c[q] * pow(2.0 * sqrt(a[p] * a[q]) / (a[p] + a[q]), l + 1.5);
    const double nc = 1.0 / sqrt(s);
    for (int p = 0; p < np; ++p)
        out[p] = nc * c[p] * pow(2.0 * a[p] / M_PI, 0.75) * pow(4.0 * a[p], 0.5 * l) /
                 sqrt(dfact_odd(2 * l - 1));
}

// ------------------------------------------------------ device kernels

struct ShellDev {
    double x, y, z;
    int prim0, nprim;
};

__global__ void k_build_pairs(int n, const int2 *__restrict__ ab, const int *__restrict__ pp0,
                              const ShellDev *__restrict__ sh, const int *__restrict__ bf0,
                              const double *__restrict__ alpha, const double *__restrict__ ct,
                              PairInfo *__restrict__ pairs, PrimPair *__restrict__ pp) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int sa = ab[i].x, sb = ab[i].y;
    const ShellDev A = sh[sa], B = sh[sb];
    PairInfo pi;
    pi.Ax = A.x; pi.Ay = A.y; pi.Az = A.z;
    pi.ABx = A.x - B.x; pi.ABy = A.y - B.y; pi.ABz = A.z - B.z;
    pi.pp0 = pp0[i];
    pi.npp = A.nprim * B.nprim;
    pi.sa = sa; pi.sb = sb;
    pi.bfa = bf0[sa]; pi.bfb = bf0[sb];
    pairs[i] = pi;
    const double ab2 = pi.ABx * pi.ABx + pi.ABy * pi.ABy + pi.ABz * pi.ABz;
    int k = pi.pp0;
    for (int u = 0; u < A.nprim; ++u) {
        const double a = alpha[A.prim0 + u], ca = ct[A.prim0 + u];
        for (int v = 0; v < B.nprim; ++v, ++k) {
            const double b = alpha[B.prim0 + v], cb = ct[B.prim0 + v];
            const double p = a + b, rp = 1.0 / p;
            PrimPair q;
            q.PAx = -b * rp * pi.ABx;
            q.PAy = -b * rp * pi.ABy;
            q.PAz = -b * rp * pi.ABz;
            q.p = p;
            q.K = ca * cb * exp(-a * b * rp * ab2);
            q.rp = rp;
            q.pad0 = q.pad1 = 0.0;
            pp[k] = q;
        }
    }
}

// Rank of each pair within its class by descending Q (ties by index);
// perm[off + rank] = local index.
__global__ void k_rank_desc(const double *__restrict__ Q, int off, int n, int *__restrict__ perm) {
    __shared__ double tile[256];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const double qi = i < n ? Q[off + i] : 0.0;
    int rank = 0;
    for (int j0 = 0; j0 < n; j0 += 256) {
        const int j = j0 + threadIdx.x;
        tile[threadIdx.x] = j < n ? Q[off + j] : 0.0;
        __syncthreads();
        const int m = min(256, n - j0);
        for (int t = 0; t < m; ++t) {
            const double qj = tile[t];
            rank += (qj > qi) || (qj == qi && j0 + t < i);
        }
        __syncthreads();
    }
    if (i < n) perm[off + rank] = i;
}

__global__ void k_gather_pairs(int off, int n, const int *__restrict__ perm,
                               const PairInfo *__restrict__ src, const double *__restrict__ Qsrc,
                               PairInfo *__restrict__ dst, double *__restrict__ Qdst) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int i = perm[off + r];
    dst[off + r] = src[off + i];
    Qdst[off + r] = Qsrc[off + i];
}

// Kets of bra row i: kets j (sorted descending) with Q_i Q_j >= tau; for a
// same-class list only j <= i.
__global__ void k_row_counts(const double *__restrict__ Q, int bra_off, int nbra, int ket_off,
                             int nket, int same_class, double tau, int64_t *__restrict__ counts) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nbra) return;
    int cnt = nket;
    if (tau > 0.0) {
        const double qi = Q[bra_off + i];
        int lo = 0, hi = nket;  // first j with qi*Q_j < tau
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (qi * Q[ket_off + mid] >= tau) lo = mid + 1; else hi = mid;
        }
        cnt = lo;
    }
    if (same_class) cnt = min(cnt, i + 1);
    counts[i] = cnt;
}

// Exclusive scan of n counts into out[0..n] with one block of 1024 threads.
__global__ void __launch_bounds__(1024) k_scan_counts(const int64_t *__restrict__ counts, int n,
                                                      int64_t *__restrict__ out) {
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int per = (n + 1023) / 1024;
    const int b = t * per, e = min(n, b + per);
    int64_t s = 0;
    for (int i = b; i < e; ++i) s += counts[i];
    part[t] = s;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const int64_t v = t >= d ? part[t - d] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t run = part[t] - s;  // exclusive prefix of this thread's segment
    for (int i = b; i < e; ++i) {
        out[i] = run;
        run += counts[i];
    }
    if (t == 1023) out[n] = part[1023];
}

// ------------------------------------------------------- host helpers

static int make_class_launch(const mess_basis *B, ClassLaunch &L, hipStream_t s) {
    L.pairs = B->d_pairs;
    L.pp = B->d_pp;
    L.ppf = B->d_ppf;
    L.tab = B->d_boys;
    L.etab = B->d_boys_exp;
    L.tabf = B->d_boys_f;
    L.etabf = B->d_boys_exp_f;
    L.N = B->nbf;
    L.stream = s;
    L.rowstart = nullptr;
    L.total = 0;
    L.bra_off = L.ket_off = L.nbra = L.same_class = 0;
    return MESS_OK;
}

int fill_class_launch(const mess_basis *B, const ClassList &cl, hipStream_t s, ClassLaunch &L) {
    make_class_launch(B, L, s);
    L.bra_off = B->pair_class_off[cl.cb];
    L.ket_off = B->pair_class_off[cl.ck];
    L.nbra = cl.nbra;
    L.same_class = cl.cb == cl.ck;
    L.rowstart = cl.d_rowstart;
    L.total = cl.total;
    return MESS_OK;
}

int get_work_lists(mess_basis *B, double tau, hipStream_t s, WorkLists **out) {
    if (!(tau > 0.0)) tau = 0.0;
    auto it = B->lists.find(tau);
    if (it != B->lists.end()) {
        *out = it->second;
        return MESS_OK;
    }
    auto *W = new WorkLists();
    W->tau = tau;
    int64_t *d_counts = nullptr;
    int maxn = 1;
    for (int c = 0; c < kNumPairClasses; ++c)
        maxn = std::max(maxn, B->pair_class_off[c + 1] - B->pair_class_off[c]);
    hipError_t e = hipMalloc(&d_counts, sizeof(int64_t) * maxn);
    if (e != hipSuccess) {
        delete W;
        set_error("hipMalloc(work-list counts) failed: %s", hipGetErrorString(e));
        return MESS_E_NOMEM;
    }
    int rc = MESS_OK;
    for (int cb = 0; cb < kNumPairClasses && rc == MESS_OK; ++cb)
        for (int ck = 0; ck <= cb && rc == MESS_OK; ++ck) {
            ClassList cl;
            cl.cb = cb;
            cl.ck = ck;
            cl.nbra = B->pair_class_off[cb + 1] - B->pair_class_off[cb];
            const int nket = B->pair_class_off[ck + 1] - B->pair_class_off[ck];
            if (cl.nbra == 0 || nket == 0) {
                cl.total = 0;
                W->classes.push_back(cl);
                continue;
            }
            if (hipMalloc(&cl.d_rowstart, sizeof(int64_t) * (cl.nbra + 1)) != hipSuccess) {
                set_error("hipMalloc(work list) failed");
                rc = MESS_E_NOMEM;
                break;
            }
            hipLaunchKernelGGL(k_row_counts, dim3((cl.nbra + 255) / 256), dim3(256), 0, s, B->d_pairQ,
                               B->pair_class_off[cb], cl.nbra, B->pair_class_off[ck], nket, cb == ck ? 1 : 0,
                               tau, d_counts);
            hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, s, d_counts, cl.nbra, cl.d_rowstart);
            cl.h_rowstart.resize(cl.nbra + 1);
            if (hipGetLastError() != hipSuccess ||
                hipMemcpyAsync(cl.h_rowstart.data(), cl.d_rowstart, sizeof(int64_t) * (cl.nbra + 1),
                               hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                hipFree(cl.d_rowstart);
                set_error("work-list construction failed on the device");
                rc = MESS_E_DEVICE;
                break;
            }
            cl.total = cl.h_rowstart[cl.nbra];
            {
                // primitive quartets: sum_i npp(bra_i) * sum_{j < count_i} npp(ket_j)
                const int boff = B->pair_class_off[cb], koff = B->pair_class_off[ck];
                std::vector<int64_t> kpre(nket + 1, 0);
                for (int j = 0; j < nket; ++j) kpre[j + 1] = kpre[j] + B->pairs_host[koff + j].npp;
                int64_t tot = 0;
                for (int i = 0; i < cl.nbra; ++i) {
                    const int64_t cnt = cl.h_rowstart[i + 1] - cl.h_rowstart[i];
                    tot += (int64_t)B->pairs_host[boff + i].npp * kpre[cnt];
                }
                cl.prim_quartets = tot;
            }
            W->classes.push_back(cl);
        }
    hipFree(d_counts);
    if (rc != MESS_OK) {
        for (auto &cl : W->classes)
            if (cl.d_rowstart) hipFree(cl.d_rowstart);
        delete W;
        return rc;
    }
    B->lists[tau] = W;
    *out = W;
    return MESS_OK;
}

static void free_basis(mess_basis *B) {
    if (!B) return;
    for (auto &kv : B->lists) {
        for (auto &cl : kv.second->classes)
            if (cl.d_rowstart) hipFree(cl.d_rowstart);
        delete kv.second;
    }
    void free_stored(mess_basis *);
    free_stored(B);
    hipFree(B->d_xyz);
    hipFree(B->d_Zd);
    hipFree(B->d_boys);
    hipFree(B->d_boys_exp);
    hipFree(B->d_boys_f);
    hipFree(B->d_boys_exp_f);
    hipFree(B->d_pairs);
    hipFree(B->d_pairQ);
    hipFree(B->d_pp);
    hipFree(B->d_ppf);
    hipFree(B->scratch_jk);
    delete B;
}

static int create_impl(int32_t n_atoms, const int32_t *Z, const double *xyz, int32_t n_shells,
                       const int32_t *shell_atom, const int32_t *shell_l, const int32_t *shell_nprim,
                       const double *exps, const double *coefs, int32_t charge, mess_basis *B) {
    if (n_atoms <= 0 || n_shells <= 0 || !Z || !xyz || !shell_atom || !shell_l || !shell_nprim || !exps ||
        !coefs) {
        set_error("mess_basis_create: NULL array or non-positive count");
        return MESS_E_ARG;
    }
    B->nat = n_atoms;
    B->nsh = n_shells;
    B->Z.assign(Z, Z + n_atoms);
    B->xyz.assign(xyz, xyz + 3 * n_atoms);
    int zsum = 0;
    for (int a = 0; a < n_atoms; ++a) {
        if (Z[a] < 0 || Z[a] > 118) {
            set_error("mess_basis_create: atomic number %d out of range", Z[a]);
            return MESS_E_ARG;
        }
        for (int x = 0; x < 3; ++x)
            if (!std::isfinite(xyz[3 * a + x])) {
                set_error("mess_basis_create: non-finite coordinate of atom %d", a);
                return MESS_E_ARG;
            }
        zsum += Z[a];
    }
    B->nelec = zsum - charge;
    if (B->nelec < 0) {
        set_error("mess_basis_create: negative electron count");
        return MESS_E_ARG;
    }
    B->nocc = B->nelec / 2;
    int nprim = 0, nbf = 0;
    B->sh_atom.resize(n_shells);
    B->sh_l.resize(n_shells);
    B->sh_np.resize(n_shells);
    B->sh_prim0.resize(n_shells);
    B->sh_bf0.resize(n_shells);
    for (int s = 0; s < n_shells; ++s) {
        if (shell_atom[s] < 0 || shell_atom[s] >= n_atoms) {
            set_error("mess_basis_create: shell %d on atom %d out of range", s, shell_atom[s]);
            return MESS_E_ARG;
        }
        if (shell_l[s] < 0 || shell_l[s] > 2) {
            set_error("mess_basis_create: shell %d has l=%d; only s, p, d (l <= 2) are built", s,
                      shell_l[s]);
            return shell_l[s] < 0 ? MESS_E_ARG : MESS_E_UNSUPPORTED;
        }
        if (shell_nprim[s] < 1 || shell_nprim[s] > 16) {
            set_error("mess_basis_create: shell %d has %d primitives (1..16 allowed)", s, shell_nprim[s]);
            return MESS_E_ARG;
        }
        B->sh_atom[s] = shell_atom[s];
        B->sh_l[s] = shell_l[s];
        B->sh_np[s] = shell_nprim[s];
        B->sh_prim0[s] = nprim;
        B->sh_bf0[s] = nbf;
        nprim += shell_nprim[s];
        nbf += ncart(shell_l[s]);
    }
    B->nbf = nbf;
    B->alpha.assign(exps, exps + nprim);
    B->ctilde.assign(nprim, 0.0);
    for (int p = 0; p < nprim; ++p)
        if (!(exps[p] > 0.0) || !std::isfinite(exps[p]) || !std::isfinite(coefs[p])) {
            set_error("mess_basis_create: primitive %d has exponent %g, coefficient %g", p, exps[p], coefs[p]);
            return MESS_E_ARG;
        }
    for (int s = 0; s < n_shells; ++s)
        normalise(B->sh_l[s], B->sh_np[s], exps + B->sh_prim0[s], coefs + B->sh_prim0[s],
                  B->ctilde.data() + B->sh_prim0[s]);
    for (int p = 0; p < nprim; ++p)
        if (!std::isfinite(B->ctilde[p])) {
            set_error("mess_basis_create: contraction of shell with primitive %d cannot be normalised", p);
            return MESS_E_ARG;
        }
    // nuclear repulsion
    double en = 0.0;
    for (int a = 0; a < n_atoms; ++a)
        for (int b = 0; b < a; ++b) {
            const double dx = xyz[3 * a] - xyz[3 * b], dy = xyz[3 * a + 1] - xyz[3 * b + 1],
                         dz = xyz[3 * a + 2] - xyz[3 * b + 2];
            const double r = sqrt(dx * dx + dy * dy + dz * dz);
            if (r == 0.0 && Z[a] * Z[b] != 0) {
                set_error("mess_basis_create: atoms %d and %d coincide", a, b);
                return MESS_E_ARG;
            }
            if (r > 0.0) en += (double)Z[a] * Z[b] / r;
        }
    B->enuc = en;
    MESS_HIP(hipGetDevice(&B->device));

    // Boys tables
    std::vector<double> tab, etab;
    build_boys_table(tab, etab);
    std::vector<float> tabf(tab.begin(), tab.end()), etabf(etab.begin(), etab.end());
    MESS_HIP(hipMalloc(&B->d_boys, sizeof(double) * tab.size()));
    MESS_HIP(hipMalloc(&B->d_boys_exp, sizeof(double) * etab.size()));
    MESS_HIP(hipMalloc(&B->d_boys_f, sizeof(float) * tabf.size()));
    MESS_HIP(hipMalloc(&B->d_boys_exp_f, sizeof(float) * etabf.size()));
    MESS_HIP(hipMemcpy(B->d_boys, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice));
    MESS_HIP(hipMemcpy(B->d_boys_exp, etab.data(), sizeof(double) * etab.size(), hipMemcpyHostToDevice));
    MESS_HIP(hipMemcpy(B->d_boys_f, tabf.data(), sizeof(float) * tabf.size(), hipMemcpyHostToDevice));
    MESS_HIP(hipMemcpy(B->d_boys_exp_f, etabf.data(), sizeof(float) * etabf.size(), hipMemcpyHostToDevice));

    // atoms
    std::vector<double> Zd(Z, Z + n_atoms);
    MESS_HIP(hipMalloc(&B->d_xyz, sizeof(double) * 3 * n_atoms));
    MESS_HIP(hipMalloc(&B->d_Zd, sizeof(double) * n_atoms));
    MESS_HIP(hipMemcpy(B->d_xyz, xyz, sizeof(double) * 3 * n_atoms, hipMemcpyHostToDevice));
    MESS_HIP(hipMemcpy(B->d_Zd, Zd.data(), sizeof(double) * n_atoms, hipMemcpyHostToDevice));

    // shell pairs (a, b) with l_a > l_b, or l_a == l_b and a >= b, grouped by class
    std::vector<std::vector<int2>> by_class(kNumPairClasses);
    for (int a = 0; a < n_shells; ++a)
        for (int b = 0; b < n_shells; ++b) {
            const int la = B->sh_l[a], lb = B->sh_l[b];
            if (la > lb || (la == lb && a >= b)) by_class[pair_class_of(la, lb)].push_back(make_int2(a, b));
        }
    std::vector<int2> pairs_ab;
    std::vector<int> pp0;
    int npp = 0;
    for (int c = 0; c < kNumPairClasses; ++c) {
        B->pair_class_off[c] = (int)pairs_ab.size();
        for (auto ab : by_class[c]) {
            pairs_ab.push_back(ab);
            pp0.push_back(npp);
            npp += B->sh_np[ab.x] * B->sh_np[ab.y];
        }
    }
    B->pair_class_off[kNumPairClasses] = (int)pairs_ab.size();
    B->npair = (int)pairs_ab.size();
    B->npp = npp;
    std::vector<ShellDev> shd(n_shells);
    for (int s = 0; s < n_shells; ++s) {
        const int a = B->sh_atom[s];
        shd[s] = ShellDev{xyz[3 * a], xyz[3 * a + 1], xyz[3 * a + 2], B->sh_prim0[s], B->sh_np[s]};
    }

    int2 *d_ab = nullptr;
    int *d_pp0 = nullptr, *d_bf0 = nullptr, *d_perm = nullptr;
    ShellDev *d_sh = nullptr;
    double *d_alpha = nullptr, *d_ct = nullptr, *d_Qraw = nullptr;
    PairInfo *d_pairs_raw = nullptr;
    int rc = MESS_OK;
    auto cleanup = [&]() {
        hipFree(d_ab); hipFree(d_pp0); hipFree(d_bf0); hipFree(d_perm); hipFree(d_sh);
        hipFree(d_alpha); hipFree(d_ct); hipFree(d_Qraw); hipFree(d_pairs_raw);
    };
#define MESS_HIPC(call)                                                                         \
    do {                                                                                        \
        hipError_t _e = (call);                                                                 \
        if (_e != hipSuccess) {                                                                 \
            set_error("%s failed: %s", #call, hipGetErrorString(_e));                           \
            cleanup();                                                                          \
            return _e == hipErrorOutOfMemory ? MESS_E_NOMEM : MESS_E_DEVICE;                    \
        }                                                                                       \
    } while (0)
    const int np_ = B->npair;
    MESS_HIPC(hipMalloc(&d_ab, sizeof(int2) * np_));
    MESS_HIPC(hipMalloc(&d_pp0, sizeof(int) * np_));
    MESS_HIPC(hipMalloc(&d_bf0, sizeof(int) * n_shells));
    MESS_HIPC(hipMalloc(&d_perm, sizeof(int) * np_));
    MESS_HIPC(hipMalloc(&d_sh, sizeof(ShellDev) * n_shells));
    MESS_HIPC(hipMalloc(&d_alpha, sizeof(double) * nprim));
    MESS_HIPC(hipMalloc(&d_ct, sizeof(double) * nprim));
    MESS_HIPC(hipMalloc(&d_Qraw, sizeof(double) * np_));
    MESS_HIPC(hipMalloc(&d_pairs_raw, sizeof(PairInfo) * np_));
    MESS_HIPC(hipMalloc(&B->d_pairs, sizeof(PairInfo) * np_));
    MESS_HIPC(hipMalloc(&B->d_pairQ, sizeof(double) * np_));
    MESS_HIPC(hipMalloc(&B->d_pp, sizeof(PrimPair) * npp));
    MESS_HIPC(hipMemcpy(d_ab, pairs_ab.data(), sizeof(int2) * np_, hipMemcpyHostToDevice));
    MESS_HIPC(hipMemcpy(d_pp0, pp0.data(), sizeof(int) * np_, hipMemcpyHostToDevice));
    MESS_HIPC(hipMemcpy(d_bf0, B->sh_bf0.data(), sizeof(int) * n_shells, hipMemcpyHostToDevice));
    MESS_HIPC(hipMemcpy(d_sh, shd.data(), sizeof(ShellDev) * n_shells, hipMemcpyHostToDevice));
    MESS_HIPC(hipMemcpy(d_alpha, exps, sizeof(double) * nprim, hipMemcpyHostToDevice));
    MESS_HIPC(hipMemcpy(d_ct, B->ctilde.data(), sizeof(double) * nprim, hipMemcpyHostToDevice));
    hipStream_t s = nullptr;
    hipLaunchKernelGGL(k_build_pairs, dim3((np_ + 127) / 128), dim3(128), 0, s, np_, d_ab, d_pp0, d_sh, d_bf0,
                       d_alpha, d_ct, d_pairs_raw, B->d_pp);
    MESS_HIPC(hipGetLastError());

    // Schwarz factors per pair (diagonal quartets), then sort each class by Q
    ClassLaunch L;
    make_class_launch(B, L, s);
    L.pairs = d_pairs_raw;
    for (int c = 0; c < kNumPairClasses && rc == MESS_OK; ++c) {
        const int off = B->pair_class_off[c], n = B->pair_class_off[c + 1] - off;
        if (n == 0) continue;
        rc = dispatch_class(c, c, [&](auto CB, auto CK) {
            return ClassOps<decltype(CB)::value, decltype(CK)::value>::schwarz(L, off, n, d_Qraw);
        });
    }
    if (rc != MESS_OK) {
        cleanup();
        return rc;
    }
    for (int c = 0; c < kNumPairClasses; ++c) {
        const int off = B->pair_class_off[c], n = B->pair_class_off[c + 1] - off;
        if (n == 0) continue;
        hipLaunchKernelGGL(k_rank_desc, dim3((n + 255) / 256), dim3(256), 0, s, d_Qraw, off, n, d_perm);
        hipLaunchKernelGGL(k_gather_pairs, dim3((n + 255) / 256), dim3(256), 0, s, off, n, d_perm, d_pairs_raw,
                           d_Qraw, B->d_pairs, B->d_pairQ);
    }
    MESS_HIPC(hipGetLastError());
    B->pairQ_host.resize(np_);
    MESS_HIPC(hipMemcpy(B->pairQ_host.data(), B->d_pairQ, sizeof(double) * np_, hipMemcpyDeviceToHost));
    B->pairs_host.resize(np_);
    MESS_HIPC(hipMemcpy(B->pairs_host.data(), B->d_pairs, sizeof(PairInfo) * np_, hipMemcpyDeviceToHost));
    for (int i = 0; i < np_; ++i)
        if (!std::isfinite(B->pairQ_host[i])) {
            set_error("mess_basis_create: non-finite Schwarz factor (pair %d)", i);
            cleanup();
            return MESS_E_NUMERIC;
        }
    // FP32 copy of the primitive-pair table
    {
        std::vector<PrimPair> h(npp);
        MESS_HIPC(hipMemcpy(h.data(), B->d_pp, sizeof(PrimPair) * npp, hipMemcpyDeviceToHost));
        std::vector<PrimPairF> hf(npp);
        for (int i = 0; i < npp; ++i)
            hf[i] = PrimPairF{(float)h[i].PAx, (float)h[i].PAy, (float)h[i].PAz, (float)h[i].p,
                              (float)h[i].K, (float)h[i].rp, 0.0f, 0.0f};
        MESS_HIPC(hipMalloc(&B->d_ppf, sizeof(PrimPairF) * npp));
        MESS_HIPC(hipMemcpy(B->d_ppf, hf.data(), sizeof(PrimPairF) * npp, hipMemcpyHostToDevice));
    }
    MESS_HIPC(hipMalloc(&B->scratch_jk, sizeof(double) * 2 * (size_t)nbf * nbf));
#undef MESS_HIPC
    cleanup();
    return MESS_OK;
}

}  // namespace mess

using namespace mess;

extern "C" {

const char *mess_last_error(void) { return g_err; }

int mess_basis_create(int32_t n_atoms, const int32_t *Z, const double *xyz_bohr, int32_t n_shells,
                      const int32_t *shell_atom, const int32_t *shell_l, const int32_t *shell_nprim,
                      const double *exps, const double *coefs, int32_t charge, mess_basis **out) {
    g_err[0] = 0;
    if (!out) {
        set_error("mess_basis_create: out is NULL");
        return MESS_E_ARG;
    }
    *out = nullptr;
    auto *B = new mess_basis();
    int rc = create_impl(n_atoms, Z, xyz_bohr, n_shells, shell_atom, shell_l, shell_nprim, exps, coefs, charge,
                         B);
    if (rc != MESS_OK) {
        free_basis(B);
        return rc;
    }
    *out = B;
    return MESS_OK;
}

void mess_basis_destroy(mess_basis *basis) { free_basis(basis); }

int mess_work_stats(const mess_basis *basis, double schwarz_tol, int32_t cls, int64_t *quartets,
                    int64_t *prim_quartets, double *alg_flops_jk) {
    if (!basis || cls < 0 || cls > 20) {
        set_error("mess_work_stats: NULL basis or class index outside 0..20");
        return MESS_E_ARG;
    }
    WorkLists *W = nullptr;
    MESS_TRY(get_work_lists(const_cast<mess_basis *>(basis), schwarz_tol, nullptr, &W));
    for (const ClassList &cl : W->classes)
        if (class_index(cl.cb, cl.ck) == cls) {
            double fp = 0.0, fq = 0.0;
            class_flops(cl.cb, cl.ck, &fp, &fq);
            if (quartets) *quartets = cl.total;
            if (prim_quartets) *prim_quartets = cl.prim_quartets;
            if (alg_flops_jk) *alg_flops_jk = fp * (double)cl.prim_quartets + fq * (double)cl.total;
            return MESS_OK;
        }
    if (quartets) *quartets = 0;
    if (prim_quartets) *prim_quartets = 0;
    if (alg_flops_jk) *alg_flops_jk = 0.0;
    return MESS_OK;
}

int mess_basis_info(const mess_basis *B, int32_t *nbf, int32_t *n_occ, double *e_nuc) {
    if (!B) {
        set_error("mess_basis_info: basis is NULL");
        return MESS_E_ARG;
    }
    if (nbf) *nbf = B->nbf;
    if (n_occ) *n_occ = B->nocc;
    if (e_nuc) *e_nuc = B->enuc;
    return MESS_OK;
}

}  // extern "C"
