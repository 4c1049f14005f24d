// Internal declarations shared by the HIP translation units of libmess_hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "../../include/mess.h"

namespace mess {

// ------------------------------------------------------------------ errors

void set_error(const char *fmt, ...);

struct Status {
    int code = MESS_OK;
};

#define MESS_HIP(call)                                                                 \
    do {                                                                               \
        hipError_t _e = (call);                                                        \
        if (_e != hipSuccess) {                                                        \
            ::mess::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(_e),   \
                              __FILE__, __LINE__);                                     \
            return (_e == hipErrorOutOfMemory) ? MESS_E_NOMEM : MESS_E_DEVICE;         \
        }                                                                              \
    } while (0)

#define MESS_TRY(expr)                     \
    do {                                   \
        int _rc = (expr);                  \
        if (_rc != MESS_OK) return _rc;    \
    } while (0)

// Launch check: catches bad launch configurations immediately.
#define MESS_LAUNCH_CHECK() MESS_HIP(hipGetLastError())

// -------------------------------------------------- compile-time loops

template <typename F, int... Is>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, Is...>) {
    (f(std::integral_constant<int, Is>{}), ...);
}

// Calls f(integral_constant<int, i>) for i in [Begin, End).
template <int Begin, int End, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (Begin < End) {
        static_for_impl(
            [&](auto i) { f(std::integral_constant<int, Begin + decltype(i)::value>{}); },
            std::make_integer_sequence<int, End - Begin>{});
    }
}

// --------------------------------------------- Cartesian component tables
//
// Components of angular momentum l are ordered x-major lexicographically:
// (l,0,0), (l-1,1,0), (l-1,0,1), (l-2,2,0), ...  A "global" index counts
// the components of all l' < l first, so every component of every
// angular momentum up to some maximum has one index.

__host__ __device__ constexpr int ncart(int l) { return (l + 1) * (l + 2) / 2; }
__host__ __device__ constexpr int cart_off(int l) { return l * (l + 1) * (l + 2) / 6; }
__host__ __device__ constexpr int cart_idx(int x, int y, int z) {
    return cart_off(x + y + z) + (y + z) * (y + z + 1) / 2 + z;
}

struct Cart {
    int x, y, z;
    __host__ __device__ constexpr int l() const { return x + y + z; }
    __host__ __device__ constexpr int get(int d) const { return d == 0 ? x : (d == 1 ? y : z); }
    // Direction used to lower this component in a recurrence: the first
    // direction with a non-zero exponent.
    __host__ __device__ constexpr int dir() const { return x > 0 ? 0 : (y > 0 ? 1 : 2); }
    __host__ __device__ constexpr Cart minus(int d, int k = 1) const {
        return Cart{x - (d == 0 ? k : 0), y - (d == 1 ? k : 0), z - (d == 2 ? k : 0)};
    }
    __host__ __device__ constexpr Cart plus(int d, int k = 1) const { return minus(d, -k); }
    __host__ __device__ constexpr int idx() const { return cart_idx(x, y, z); }
};

__host__ __device__ constexpr Cart cart_of(int idx) {
    int l = 0;
    while (cart_off(l + 1) <= idx) ++l;
    int r = idx - cart_off(l);
    int k = 0;  // k = l - lx
    while ((k + 1) * (k + 2) / 2 <= r) ++k;
    int z = r - k * (k + 1) / 2;
    return Cart{l - k, k - z, z};
}

// Ratio N(alpha; lx,ly,lz) / N(alpha; l,0,0) of primitive normalisation
// constants, i.e. sqrt((2l-1)!! / ((2lx-1)!! (2ly-1)!! (2lz-1)!!)).  For
// l <= 2 it is sqrt(3) for the mixed d components (xy, xz, yz), else 1.
__host__ __device__ constexpr bool cart_is_mixed_d(Cart c) {
    return c.l() == 2 && c.x < 2 && c.y < 2 && c.z < 2;
}
constexpr double kSqrt3 = 1.7320508075688772935;

// ------------------------------------------------------------ device data

// One shell pair (a, b) with l_a >= l_b.  A is the centre of shell a,
// AB = A - B.  Primitive pairs live in pp[pp0 .. pp0 + npp).
struct PairInfo {
    double Ax, Ay, Az;
    double ABx, ABy, ABz;
    int pp0, npp;
    int sa, sb;    // shell indices
    int bfa, bfb;  // first basis function of each shell, within its molecule
    int moff, mN;  // packed-matrix offset and dimension of the molecule
};

// One primitive pair (alpha on A, beta on B): p = alpha + beta,
// PA = P - A = -(beta/p) AB (computed from AB so it is exactly zero when
// both shells sit on one atom), K = c_a c_b exp(-alpha beta/p |AB|^2) with
// c the normalised contraction coefficients of the l,0,0 component.
// The Gaussian product centre is P = A + PA.
struct PrimPair {
    double PAx, PAy, PAz, p;
    double K, rp, Kr, pad1;  // rp = 1/p, Kr = sqrt(2 pi^{5/2}) K / p
};

struct PrimPairF {
    float PAx, PAy, PAz, p;
    float K, rp, Kr, pad1;
};

// Boys table: F_n(T_k), n = 0..kBoysN-1, T_k = k / kBoysInvStep, T_k <= kBoysTmax.
constexpr int kBoysN = 16;
constexpr double kBoysInvStep = 16.0;
constexpr double kBoysTmax = 60.0;
constexpr int kBoysRows = 961;  // kBoysTmax * kBoysInvStep + 1
// Taylor table per order L = 0..kBoysTL-1: row k holds F_{L+i}(T_k) / i!, i < 8.
constexpr int kBoysTL = kBoysN - 7;

// Pair classes (l_a, l_b), l_a >= l_b: ss ps pp ds dp dd.
constexpr int kNumPairClasses = 6;
__host__ __device__ constexpr int pair_class_la(int c) { return c == 0 ? 0 : (c <= 2 ? 1 : 2); }
__host__ __device__ constexpr int pair_class_lb(int c) {
    return c == 0 ? 0 : (c == 1 ? 0 : (c == 2 ? 1 : (c == 3 ? 0 : (c == 4 ? 1 : 2))));
}
inline int pair_class_of(int la, int lb) {
    // la >= lb
    if (la == 0) return 0;
    if (la == 1) return lb == 0 ? 1 : 2;
    return lb == 0 ? 3 : (lb == 1 ? 4 : 5);
}

// Unique shell-quartet work list of one class: bra pairs of class cb and
// ket pairs of class ck (cb >= ck).  Within each (class, molecule) segment
// the pairs are sorted by primitive-pair count (descending), then by
// Schwarz factor (descending), so a segment is a run of buckets of equal
// primitive count, each sorted by Q.  The kets of bra i that pass
// screening form a prefix of every bucket; the list holds one row per
// (bra, bucket) with a non-empty prefix: rowmap[r] = {bra index, first ket
// index}, both relative to their class, and the row's quartets are
// [rowstart[r], rowstart[r + 1]) with ket index = first ket + (t -
// rowstart[r]).  Lanes of a wave taking consecutive quartets then see
// kets of (nearly) equal primitive count.
struct ClassList {
    int cb, ck;
    int nbra;                         // bra pairs of the class
    int nrow = 0;                     // rows of the list
    int64_t total = 0;                // shell quartets
    int64_t prim_quartets = 0;        // sum over quartets of (bra prim pairs) x (ket prim pairs)
    int64_t *d_rowstart = nullptr;    // nrow + 1
    int2 *d_rowmap = nullptr;         // nrow
    std::vector<int64_t> h_rowstart;  // host copies
    std::vector<int2> h_rowmap;
    // the quartets of each bra (its consecutive rows) in pieces of at most
    // kSegLen: {first row, first quartet, end quartet, end row}; NULL when
    // the list has 2^31 quartets or more
    int4 *d_segs = nullptr;
    int nseg = 0;
    // groups of kGroupBras[cb] consecutive bras of one molecule for the
    // grouped stored digestion: per group {first tile, end tile, first bra,
    // bras}; per tile (one ket bucket of the group) {offset of its
    // kGroupBras[cb] row indices in d_grows (-1: no row), first ket index,
    // longest row, ket offset of the tile within its group}; NULL when
    // kGroupBras[cb] is 1 or the list has 2^31 quartets or more
    int4 *d_groups = nullptr, *d_tiles = nullptr;
    int *d_grows = nullptr;
    int ngroups = 0;
};
constexpr int64_t kSegLen = 512;
// bras per group of the grouped stored digestion, by bra pair class (ss ps
// pp ds dp dd), within 48 KB of LDS for the group's exchange rows (NA + NB
// rows per bra) at 300 functions; 1: by segments.  Measured per build on
// the 60-atom cluster (segments -> groups): (ss|ss) 0.91 -> 0.30 ms, (ps|ss)
// 0.57 -> 0.30, (ds|ss) 0.61 -> 0.47, (ds|ds) 0.46 -> 0.30; pp bras in
// threes and dp bras in pairs ran slower ((pp|ss) 0.09 -> 0.20, (dp|ds)
// 0.24 -> 0.34: fewer blocks per CU fit the larger LDS rows)
constexpr int kGroupBras[6] = {8, 4, 1, 2, 1, 1};

// Index 0..20 of the class (cb >= ck).
inline int class_index(int cb, int ck) { return cb * (cb + 1) / 2 + ck; }

// Algorithmic FP64 operation counts of the recursion for one class (an FMA
// counts 2): per primitive quartet (Boys, vertical recursion, contraction)
// and per shell quartet (horizontal recursion + J/K digestion).
void class_flops(int cb, int ck, double *per_prim, double *per_quartet_jk, int prec = MESS_FP64);

// True when class (cb, ck) has nothing left to allocate on the device for
// its launches (cooperative step tables built, or none needed).
bool coop_program_cached(int cb, int ck);
// Classes evaluated by the wave-per-quartet kernels (coop.hip, plane.hip).
bool coop_class(int cb, int ck);

// Kernel form of a class (tune.hip): the mapping of its quartets onto the
// hardware.  Values match the MESS_FORM_* constants of the C ABI.
enum : int { kFormAuto = 0, kFormLane = 1, kFormRows = 2, kFormPlane = 3, kFormCoop = 4, kFormWave = 5,
             kFormFp64 = 6, kNumForms = 7 };
// kFormFp64 (FP32 table only): builds asked for in FP32 evaluate the class in
// FP64 arithmetic, with its FP64 form (where that kernel is the faster one).
constexpr int kNumClasses = 21;
int class_form(int cb, int ck, int prec = MESS_FP64);  // active form (built-in default unless set)
bool form_valid(int cb, int ck, int form, int prec = MESS_FP64);
bool plane_compiled(int cb, int ck);  // primitive-lane kernel built for the class
bool wave_compiled(int cb, int ck);   // wave-per-primitive-quartet kernel built for the class
bool rows_compiled(int cb, int ck);   // bra-segment kernel built for the class

// Profiling of class launches (HIP events on the launch stream).
bool prof_on();
void prof_record(hipStream_t s, int cls, bool begin, int64_t quartets, int64_t prims, double flops);

struct WorkLists {
    double tau = -1.0;
    std::vector<ClassList> classes;  // 21 (cb >= ck), in a fixed order
    void *dbuf = nullptr;            // one device allocation holding every class's lists
};

struct StoredEri;  // mess_jk(STORED) cache

}  // namespace mess

struct mess_basis {
    int nat = 0, nsh = 0, nbf = 0, nelec = 0, nocc = 0;
    double enuc = 0.0;
    // Batches of molecules (a single molecule is a batch of one): functions
    // are numbered molecule by molecule; matrices are packed block-diagonal,
    // molecule m's nbf_m x nbf_m block at offset mol_moff[m].
    int n_mol = 1;
    std::vector<int> mol_atom0, mol_natom, mol_sh0, mol_nsh, mol_bf0, mol_nbf, mol_nelec, mol_nocc;
    std::vector<int64_t> mol_moff;  // n_mol + 1
    std::vector<double> mol_enuc;
    int64_t packed = 0;             // sum of nbf_m^2
    int64_t *d_mol_moff = nullptr;  // device copies: n_mol + 1 offsets, n_mol dimensions
    int *d_mol_nbf = nullptr;
    int nbf_max = 0;
    std::vector<int> seg_off[mess::kNumPairClasses], seg_cnt[mess::kNumPairClasses];  // per molecule
    std::vector<int> Z, sh_atom, sh_l, sh_np, sh_prim0, sh_bf0;
    std::vector<double> xyz, alpha, ctilde;  // ctilde: normalised coefs (l,0,0)
    int device = 0;

    // device tables
    double *d_xyz = nullptr;   // [nat*3]
    double *d_Zd = nullptr;    // [nat] charges as double
    double *d_boys = nullptr;  // [kBoysRows * kBoysN]
    double *d_boys_exp = nullptr;  // [kBoysRows]: exp(-T_k)
    double *d_boys_t = nullptr;    // [kBoysTL][kBoysRows][8]: F_{L+i}(T_k) / i!
    float *d_boys_f = nullptr;     // FP32 copy of the table
    float *d_boys_exp_f = nullptr;

    int npair = 0;
    int pair_class_off[mess::kNumPairClasses + 1] = {0};
    mess::PairInfo *d_pairs = nullptr;     // sorted by class, then Q descending
    double *d_pairQ = nullptr;             // Schwarz factor per sorted pair
    mess::PrimPair *d_pp = nullptr;        // primitive pairs (unsorted)
    mess::PrimPairF *d_ppf = nullptr;      // FP32 copy
    int npp = 0;            // primitive pairs kept after screening
    int64_t npp_full = 0;   // before screening
    std::vector<double> pairQ_host;        // for diagnostics
    std::vector<mess::PairInfo> pairs_host;  // sorted pairs (host copy)

    std::map<double, mess::WorkLists *> lists;  // keyed by tau
    std::map<std::pair<int, double>, mess::StoredEri *> stored;  // (prec, tau)
    void *scratch_jk = nullptr;   // [2 * packed] doubles: Gj, Gk
    void *det_acc = nullptr;      // deterministic J/K: 128-bit accumulators (built on first use)
    void *xc = nullptr;           // LDA grid and basis values (built on first use)
    void *guess = nullptr;        // learned-guess pair tables (built on first use)
};
