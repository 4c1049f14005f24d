// One-electron integrals: overlap S (paper eq. 3), kinetic T and nuclear
// attraction V, one wave per ordered shell pair (pairs listed per angular
// class, one launch per class), its lanes over the molecule's nuclei.
//   1-D overlaps (Obara-Saika):  s_{00} = sqrt(pi/p),
//     s_{i+1,j} = PA s_{ij} + (i s_{i-1,j} + j s_{i,j-1}) / (2p),
//     s_{i,j+1} = PB s_{ij} + (i s_{i-1,j} + j s_{i,j-1}) / (2p);
//   kinetic, from -1/2 d^2/dx^2 acting on the ket factor:
//     t_{ij} = -2 b^2 s_{i,j+2} + b (2j+1) s_{ij} - j(j-1)/2 s_{i,j-2};
//   nuclear attraction (Obara-Saika), per nucleus C:
//     [e+1_i]^(m) = PA_i [e]^(m) - PC_i [e]^(m+1) + e_i/(2p) ([e-1_i]^(m) - [e-1_i]^(m+1)),
//     [0]^(m) = 2 pi / p  K_ab F_m(p |PC|^2),  then the HRR to (a|b).
#include <algorithm>

#include "eri_hgp.hpp"
#include "mess_internal.hpp"

namespace mess {

struct ShellLite {
    double x, y, z;
    int l, prim0, nprim, bf0;  // bf0 within the molecule
    int moff, mN;              // packed block of the molecule
    int at0, nat;              // the molecule's nuclei
};

// Every lane forms the pair's overlap and kinetic sums (lane 0 stores
// them); lane k takes nuclei k, k + 64, ... of the nuclear attraction, whose
// e-side sums are added over the wave before the horizontal recursion.
template <int LA, int LB>
__global__ void __launch_bounds__(64) k_one_electron(int npairs, const int2 *__restrict__ ab,
                                                     const ShellLite *__restrict__ sh,
                                                     const double *__restrict__ alpha,
                                                     const double *__restrict__ ct,
                                                     const double *__restrict__ xyz,
                                                     const double *__restrict__ Zc,
                                                     const double *__restrict__ tab,
                                                     const double *__restrict__ etab,
                                                     double *__restrict__ S, double *__restrict__ T,
                                                     double *__restrict__ V) {
    const int lane = threadIdx.x;
    for (int t = blockIdx.x; t < npairs; t += gridDim.x) {
    const int2 q = ab[t];
    const ShellLite A = sh[q.x], B = sh[q.y];
    const int N = A.mN;
    constexpr int NA = ncart(LA), NB = ncart(LB), LAB = LA + LB;
    constexpr int E0 = cart_off(LA), NE = cart_off(LAB + 1);
    const double AB[3] = {A.x - B.x, A.y - B.y, A.z - B.z};
    const double ab2 = AB[0] * AB[0] + AB[1] * AB[1] + AB[2] * AB[2];
    double sacc[NA * NB], tacc[NA * NB], vacc[NE - E0];
    static_for<0, NA * NB>([&](auto I) { sacc[I] = 0.0; tacc[I] = 0.0; });
    static_for<0, NE - E0>([&](auto I) { vacc[I] = 0.0; });
    for (int u = 0; u < A.nprim; ++u) {
        const double a = alpha[A.prim0 + u];
        for (int v = 0; v < B.nprim; ++v) {
            const double b = alpha[B.prim0 + v];
            const double p = a + b, rp = 1.0 / p, o2p = 0.5 * rp;
            const double K = ct[A.prim0 + u] * ct[B.prim0 + v] * exp(-a * b * rp * ab2);
            // P - A and P - B from AB, exactly zero when A = B
            const double PA[3] = {-b * rp * AB[0], -b * rp * AB[1], -b * rp * AB[2]};
            const double PB[3] = {a * rp * AB[0], a * rp * AB[1], a * rp * AB[2]};
            // 1-D overlaps s[x][i][j], i <= LA, j <= LB + 2
            double s[3][LA + 1][LB + 3];
            static_for<0, 3>([&](auto X) {
                constexpr int x = decltype(X)::value;
                s[x][0][0] = sqrt(M_PI * rp);
                static_for<1, LA + 1>([&](auto I) {
                    constexpr int i = decltype(I)::value;
                    double w = PA[x] * s[x][i - 1][0];
                    if constexpr (i >= 2) w += (i - 1) * o2p * s[x][i - 2][0];
                    s[x][i][0] = w;
                });
                static_for<0, LA + 1>([&](auto I) {
                    constexpr int i = decltype(I)::value;
                    static_for<1, LB + 3>([&](auto J) {
                        constexpr int j = decltype(J)::value;
                        double w = PB[x] * s[x][i][j - 1];
                        if constexpr (i >= 1) w += i * o2p * s[x][i - 1][j - 1];
                        if constexpr (j >= 2) w += (j - 1) * o2p * s[x][i][j - 2];
                        s[x][i][j] = w;
                    });
                });
            });
            static_for<0, NA>([&](auto IA) {
                static_for<0, NB>([&](auto IB) {
                    constexpr Cart ca = cart_of(E0 + decltype(IA)::value);
                    constexpr Cart cb = cart_of(cart_off(LB) + decltype(IB)::value);
                    double sd[3], td[3];
                    static_for<0, 3>([&](auto X) {
                        constexpr int x = decltype(X)::value;
                        constexpr int i = ca.get(x), j = cb.get(x);
                        sd[x] = s[x][i][j];
                        double k = -2.0 * b * b * s[x][i][j + 2] + b * (2 * j + 1) * s[x][i][j];
                        if constexpr (j >= 2) k -= 0.5 * j * (j - 1) * s[x][i][j - 2];
                        td[x] = k;
                    });
                    constexpr int o = decltype(IA)::value * NB + decltype(IB)::value;
                    sacc[o] += K * sd[0] * sd[1] * sd[2];
                    tacc[o] += K * (td[0] * sd[1] * sd[2] + sd[0] * td[1] * sd[2] + sd[0] * sd[1] * td[2]);
                });
            });
            // nuclear attraction
            for (int c = A.at0 + lane; c < A.at0 + A.nat; c += 64) {
                const double PC[3] = {(A.x - xyz[3 * c]) + PA[0], (A.y - xyz[3 * c + 1]) + PA[1],
                                      (A.z - xyz[3 * c + 2]) + PA[2]};
                const double Tb = p * (PC[0] * PC[0] + PC[1] * PC[1] + PC[2] * PC[2]);
                double F[LAB + 1];
                boys_f64<LAB>(Tb, tab, etab, F);
                const double pre = -Zc[c] * 2.0 * M_PI * rp * K;
                double w[NE][LAB + 1];
                static_for<0, LAB + 1>([&](auto M) { w[0][M] = pre * F[M]; });
                static_for<1, NE>([&](auto EI) {
                    constexpr int e = decltype(EI)::value;
                    constexpr Cart ce = cart_of(e);
                    constexpr int i = ce.dir();
                    constexpr int ei = ce.get(i);
                    constexpr int e1 = ce.minus(i).idx();
                    static_for<0, LAB - ce.l() + 1>([&](auto M) {
                        constexpr int m = decltype(M)::value;
                        double val = PA[i] * w[e1][m] - PC[i] * w[e1][m + 1];
                        if constexpr (ei >= 2) {
                            constexpr int e2 = ce.minus(i, 2).idx();
                            val += (ei - 1) * o2p * (w[e2][m] - w[e2][m + 1]);
                        }
                        w[e][m] = val;
                    });
                });
                static_for<E0, NE>([&](auto EI) { vacc[EI - E0] += w[EI][0]; });
            }
        }
    }
    static_for<0, NE - E0>([&](auto I) {
        for (int off = 32; off > 0; off >>= 1) vacc[I] += __shfl_xor(vacc[I], off, 64);
    });
    if (lane == 0) {
        double vout[NA * NB];
        hrr_1<LA, LB>(vacc, AB, vout);
        static_for<0, NA>([&](auto IA) {
            static_for<0, NB>([&](auto IB) {
                constexpr int ia = decltype(IA)::value, ib = decltype(IB)::value;
                constexpr double sc = comp_scale<LA>(ia) * comp_scale<LB>(ib);
                const int64_t idx = A.moff + (int64_t)(A.bf0 + ia) * N + B.bf0 + ib;
                if (S) S[idx] = sc * sacc[ia * NB + ib];
                if (T) T[idx] = sc * tacc[ia * NB + ib];
                if (V) V[idx] = sc * vout[ia * NB + ib];
            });
        });
    }
    }
}

}  // namespace mess

using namespace mess;

extern "C" int mess_one_electron(const mess_basis *B, double *S, double *T, double *V, mess_stream stream) {
    if (!B) {
        set_error("mess_one_electron: basis is NULL");
        return MESS_E_ARG;
    }
    if (!S && !T && !V) return MESS_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<ShellLite> h(B->nsh);
    std::vector<int2> by_class[9];  // ordered pairs by (l_a, l_b)
    for (int m = 0; m < B->n_mol; ++m) {
        const int s0 = B->mol_sh0[m], s1 = s0 + B->mol_nsh[m];
        for (int i = s0; i < s1; ++i) {
            const int a = B->sh_atom[i];
            h[i] = ShellLite{B->xyz[3 * a],         B->xyz[3 * a + 1],     B->xyz[3 * a + 2], B->sh_l[i],
                             B->sh_prim0[i],        B->sh_np[i],           B->sh_bf0[i] - B->mol_bf0[m],
                             (int)B->mol_moff[m],   B->mol_nbf[m],         B->mol_atom0[m],   B->mol_natom[m]};
            for (int j = s0; j < s1; ++j) by_class[3 * B->sh_l[i] + B->sh_l[j]].push_back(make_int2(i, j));
        }
    }
    std::vector<int2> pairs;
    int coff[10] = {0};
    for (int c = 0; c < 9; ++c) {
        pairs.insert(pairs.end(), by_class[c].begin(), by_class[c].end());
        coff[c + 1] = (int)pairs.size();
    }
    const int npairs = (int)pairs.size();
    int2 *d_ab = nullptr;
    ShellLite *d_sh = nullptr;
    double *d_alpha = nullptr, *d_ct = nullptr;
    const size_t np = B->alpha.size();
    int rc = MESS_OK;
    if (hipMalloc(&d_ab, sizeof(int2) * npairs) != hipSuccess || hipMalloc(&d_sh, sizeof(ShellLite) * B->nsh) != hipSuccess || hipMalloc(&d_alpha, sizeof(double) * np) != hipSuccess ||
        hipMalloc(&d_ct, sizeof(double) * np) != hipSuccess) {
        set_error("mess_one_electron: device allocation failed");
        rc = MESS_E_NOMEM;
    }
    if (rc == MESS_OK &&
        (hipMemcpyAsync(d_ab, pairs.data(), sizeof(int2) * npairs, hipMemcpyHostToDevice, s) != hipSuccess ||
         hipMemcpyAsync(d_sh, h.data(), sizeof(ShellLite) * B->nsh, hipMemcpyHostToDevice, s) != hipSuccess ||
         hipMemcpyAsync(d_alpha, B->alpha.data(), sizeof(double) * np, hipMemcpyHostToDevice, s) != hipSuccess ||
         hipMemcpyAsync(d_ct, B->ctilde.data(), sizeof(double) * np, hipMemcpyHostToDevice, s) != hipSuccess)) {
        set_error("mess_one_electron: host-to-device copy failed");
        rc = MESS_E_DEVICE;
    }
    if (rc == MESS_OK) {
#define MESS_ONEE(la, lb)                                                                                     \
    if (const int n = coff[3 * la + lb + 1] - coff[3 * la + lb])                                               \
        hipLaunchKernelGGL((k_one_electron<la, lb>), dim3((unsigned)std::min(n, 1 << 20)), dim3(64), 0, s, n,     \
                           d_ab + coff[3 * la + lb], d_sh, d_alpha, d_ct, B->d_xyz, B->d_Zd, B->d_boys,            \
                           B->d_boys_exp, S, T, V);
        MESS_ONEE(0, 0) MESS_ONEE(0, 1) MESS_ONEE(0, 2)
        MESS_ONEE(1, 0) MESS_ONEE(1, 1) MESS_ONEE(1, 2)
        MESS_ONEE(2, 0) MESS_ONEE(2, 1) MESS_ONEE(2, 2)
#undef MESS_ONEE
        if (hipGetLastError() != hipSuccess) {
            set_error("mess_one_electron: launch failed");
            rc = MESS_E_DEVICE;
        }
        // the temporaries must outlive the kernels
        if (hipStreamSynchronize(s) != hipSuccess) {
            set_error("mess_one_electron: device error");
            rc = MESS_E_DEVICE;
        }
    }
    hipFree(d_ab);
    hipFree(d_sh);
    hipFree(d_alpha);
    hipFree(d_ct);
    return rc;
}
