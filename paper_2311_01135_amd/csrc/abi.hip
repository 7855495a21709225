// C ABI of libks.so: host preparation of a batch (basis, shell pairs, quartet
// classes, grid nodes, work items), device memory layout, and the SCF driver.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "kernels.h"

namespace ks {

// ---------------------------------------------------------------------------
// errors and timing
// ---------------------------------------------------------------------------
static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

KTimer::KTimer(ks_batch* b_, const char* n, hipStream_t s_) : b(b_), name(n), s(s_)
{
    if (b->timing) {
        (void)hipEventCreate(&e0);
        (void)hipEventCreate(&e1);
        (void)hipEventRecord(e0, s);
    }
}

// Events are recorded on the batch stream around each launch and read back
// lazily (resolve_timers), so timing adds no host synchronisation.
KTimer::~KTimer()
{
    if (!b->timing) return;
    (void)hipEventRecord(e1, s);
    int idx = -1;
    for (size_t i = 0; i < b->tnames.size(); i++)
        if (b->tnames[i] == name) idx = (int)i;
    if (idx < 0) {
        idx = (int)b->tnames.size();
        b->tnames.push_back(name);
        b->tms.push_back(0.0);
        b->tms.push_back(0.0);
    }
    b->pending.push_back(ks_batch::Pending{idx, e0, e1});
}

void resolve_timers(ks_batch* b)
{
    for (auto& p : b->pending) {
        (void)hipEventSynchronize(p.e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, p.e0, p.e1);
        b->tms[2 * p.name] += ms;
        b->tms[2 * p.name + 1] += 1.0;
        (void)hipEventDestroy(p.e0);
        (void)hipEventDestroy(p.e1);
    }
    b->pending.clear();
}

// ---------------------------------------------------------------------------
// STO-3G (Hehre, Stewart, Pople 1969): universal zeta = 1 Gaussian expansions,
// scaled per element and shell by zeta^2.
// ---------------------------------------------------------------------------
struct Sto3g {
    double a1s[3] = {2.227660584, 0.4057711562, 0.1098175104};
    double d1s[3] = {0.1543289673, 0.5353281423, 0.4446345422};
    double a2sp[3] = {0.9942027, 0.2310313, 0.0751386};
    double d2s[3] = {-0.09996723, 0.39951283, 0.70011547};
    double d2p[3] = {0.15591627, 0.60768372, 0.39195739};
};

static bool element_zetas(int Z, double& z1s, double& z2sp)
{
    switch (Z) {
    case 1: z1s = 1.24; z2sp = 0.0; return true;
    case 6: z1s = 5.67; z2sp = 1.72; return true;
    case 7: z1s = 6.67; z2sp = 1.95; return true;
    case 8: z1s = 7.66; z2sp = 2.25; return true;
    case 9: z1s = 8.65; z2sp = 2.55; return true;
    default: return false;
    }
}

// 6-31G (Hehre, Ditchfield, Pople 1972; H: the 31G set), H, C, N, O: per
// heavy element a six-primitive 1s, an sp shell of three primitives (s and p
// coefficients on shared exponents) and a one-primitive outer sp shell.
struct G631Heavy {
    double a1s[6], d1s[6];
    double asp[3], ds[3], dp[3];
    double aout;
};
static const G631Heavy kG631[3] = {   // C, N, O
    {{3047.5249, 457.36951, 103.94869, 29.210155, 9.2866630, 3.1639270},
     {0.0018347, 0.0140373, 0.0688426, 0.2321844, 0.4679413, 0.3623120},
     {7.8682724, 1.8812885, 0.5442493}, {-0.1193324, -0.1608542, 1.1434564}, {0.0689991, 0.3164240, 0.7443083},
     0.1687144},
    {{4173.5110, 627.45790, 142.90210, 40.234330, 12.820210, 4.3904370},
     {0.0018348, 0.0139950, 0.0685870, 0.2322410, 0.4690700, 0.3604550},
     {11.626358, 2.7162800, 0.7722180}, {-0.1149610, -0.1691180, 1.1458520}, {0.0675800, 0.3239070, 0.7408950},
     0.2120313},
    {{5484.6717, 825.23495, 188.04696, 52.964500, 16.897570, 5.7996353},
     {0.0018311, 0.0139501, 0.0684451, 0.2327143, 0.4701930, 0.3585209},
     {15.539616, 3.5999336, 1.0137618}, {-0.1107775, -0.1480263, 1.1307670}, {0.0708743, 0.3397528, 0.7271586},
     0.2700058}};
static const double kG631H_a[3] = {18.7311370, 2.8253937, 0.6401217};
static const double kG631H_d[3] = {0.03349460, 0.23472695, 0.81375733};
static const double kG631H_aout = 0.1612778;

static int g631_heavy(int Z) { return Z == 6 ? 0 : (Z == 7 ? 1 : (Z == 8 ? 2 : -1)); }

// n primitives a0[k] zeta^2 with coefficients d[k] x primitive norms,
// renormalised so <phi|phi> = 1
static void make_shell(Shell& s, int L, int n, const double* a0, double zeta, const double* d)
{
    s.L = L;
    s.np = n;
    for (int k = 0; k < kPrimMax; k++) s.a[k] = s.c[k] = 0.0;
    for (int k = 0; k < n; k++) {
        s.a[k] = a0[k] * zeta * zeta;
        const double nk = std::pow(2.0 * s.a[k] / kPi, 0.75) * (L ? 2.0 * std::sqrt(s.a[k]) : 1.0);
        s.c[k] = d[k] * nk;
    }
    double norm = 0.0;
    for (int k = 0; k < n; k++)
        for (int l = 0; l < n; l++) {
            const double p = s.a[k] + s.a[l];
            norm += s.c[k] * s.c[l] * std::pow(kPi / p, 1.5) * (L ? 0.5 / p : 1.0);
        }
    for (int k = 0; k < n; k++) s.c[k] /= std::sqrt(norm);
}

// Appends the shells of one atom (position already in s.A, s.atom set);
// returns the number of functions added.  Guess occupations per function:
// STO-3G H 1s 1, heavy 1s 2, 2s 2, 2p (Z-4)/3; 6-31G the valence occupation
// split evenly over the inner and outer shells.
static int add_atom_shells(std::vector<Shell>& out, Shell s, int z, int basis, int nbf)
{
    const Sto3g sto;
    const int first = nbf;
    auto push = [&](int L, int n, const double* a0, double zeta, const double* d, double occ) {
        make_shell(s, L, n, a0, zeta, d);
        s.occ = occ;
        s.ao = nbf;
        out.push_back(s);
        nbf += L ? 3 : 1;
    };
    const double one = 1.0;
    if (basis == KS_BASIS_STO3G) {
        double z1, z2;
        element_zetas(z, z1, z2);
        push(0, 3, sto.a1s, z1, sto.d1s, z == 1 ? 1.0 : 2.0);
        if (z > 1) {
            push(0, 3, sto.a2sp, z2, sto.d2s, 2.0);
            push(1, 3, sto.a2sp, z2, sto.d2p, (z - 4) / 3.0);
        }
    } else if (z == 1) {
        push(0, 3, kG631H_a, 1.0, kG631H_d, 0.5);
        push(0, 1, &kG631H_aout, 1.0, &one, 0.5);
    } else {
        const G631Heavy& e = kG631[g631_heavy(z)];
        push(0, 6, e.a1s, 1.0, e.d1s, 2.0);
        push(0, 3, e.asp, 1.0, e.ds, 1.0);
        push(1, 3, e.asp, 1.0, e.dp, (z - 4) / 6.0);
        push(0, 1, &e.aout, 1.0, &one, 1.0);
        push(1, 1, &e.aout, 1.0, &one, (z - 4) / 6.0);
    }
    return nbf - first;
}

// Treutler-Ahlrichs M4 (xi = 1, alpha = 0.6) on Chebyshev nodes of the 2nd kind:
// r = (1/ln2)(1+x)^0.6 ln(2/(1-x)), w = pi/(n+1) sin(theta_i) dr/dx r^2.
static void radial_rule(int n, std::vector<double>& out)
{
    out.assign(2 * n, 0.0);
    const double al = 0.6, il2 = 1.0 / std::log(2.0);
    for (int i = 1; i <= n; i++) {
        const double th = i * kPi / (n + 1), x = std::cos(th);
        const double lg = std::log(2.0 / (1.0 - x));
        const double r = il2 * std::pow(1.0 + x, al) * lg;
        const double drdx = il2 * (al * std::pow(1.0 + x, al - 1.0) * lg + std::pow(1.0 + x, al) / (1.0 - x));
        out[i - 1] = r;
        out[n + i - 1] = kPi / (n + 1) * std::sin(th) * drdx * r * r;
    }
}

// Gauss-Legendre nodes in cos(theta) by Newton's method on the three-term
// recurrence; weights 2 / ((1 - x^2) P_n'(x)^2).
static void gauss_legendre(int n, std::vector<double>& out)
{
    out.assign(2 * n, 0.0);
    for (int i = 0; i < n; i++) {
        long double x = std::cos(kPi * (i + 0.75) / (n + 0.5)), dp = 1.0L;
        for (int it = 0; it < 200; it++) {
            long double p0 = 1.0L, p1 = x;
            for (int k = 2; k <= n; k++) {
                const long double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p0 = 1.0L; p1 = x; }
            dp = n * (x * p1 - p0) / (x * x - 1.0L);
            const long double dx = p1 / dp;
            x -= dx;
            if (std::fabs((double)dx) < 1e-19) break;
        }
        {
            long double p0 = 1.0L, p1 = x;
            for (int k = 2; k <= n; k++) {
                const long double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p0 = 1.0L; p1 = x; }
            dp = n * (x * p1 - p0) / (x * x - 1.0L);
        }
        out[i] = (double)x;
        out[n + i] = (double)(2.0L / ((1.0L - x * x) * dp * dp));
    }
}

}  // namespace ks

using namespace ks;

// ---------------------------------------------------------------------------
// allocation helpers
// ---------------------------------------------------------------------------
template <typename T>
static ks_status dev_alloc(ks_batch* b, T** p, size_t n)
{
    *p = nullptr;
    if (n == 0) n = 1;
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, n * sizeof(T));
    if (e != hipSuccess) {
        set_error("hipMalloc(%zu bytes) failed: %s", n * sizeof(T), hipGetErrorString(e));
        (void)hipGetLastError();
        return e == hipErrorOutOfMemory ? KS_ENOMEM : KS_EDEVICE;
    }
    b->allocs.push_back(q);
    b->alloc_bytes += n * sizeof(T);
    *p = (T*)q;
    return KS_OK;
}

template <typename T>
static ks_status upload(ks_batch* b, T** p, const std::vector<T>& v)
{
    ks_status st = dev_alloc(b, p, v.size());
    if (st) return st;
    if (!v.empty()) KS_HIP(hipMemcpyAsync(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, b->stream));
    return KS_OK;
}

// Integral-direct builds visit, for each bra, only the kets that pass the
// density-weighted Schwarz test; with every molecule's pairs of a class in
// decreasing order of Q (the same order for bras and kets), those kets form
// a prefix of the bra's ket range.  Reorders the pair lists, their AO
// offsets, Schwarz factors and primitive-pair tables once, after Q is known.
ks_status ks::sort_pairs_by_schwarz(ks_batch* b)
{
    if (b->pairs_sorted) return KS_OK;
    for (int c = 0; c < 3; c++) {
        const long n = b->npairs[c];
        if (!n) continue;
        std::vector<double> Q(n);
        KS_HIP(hipMemcpyAsync(Q.data(), b->d_Q[c], sizeof(double) * n, hipMemcpyDeviceToHost, b->stream));
        KS_HIP(hipStreamSynchronize(b->stream));
        std::vector<int> perm(n);
        for (long k = 0; k < n; k++) perm[k] = (int)k;
        for (const MolDesc& md : b->mol) {
            auto first = perm.begin() + md.pair0[c];
            std::stable_sort(first, first + md.npair[c], [&](int x, int y) { return Q[x] > Q[y]; });
        }
        int* d_perm;
        Pair* pairs;
        int2* pao;
        double *pp, *Qn;
        ks_status st;
        if ((st = upload(b, &d_perm, perm))) return st;
        if ((st = dev_alloc(b, &pairs, n))) return st;
        if ((st = dev_alloc(b, &pao, n))) return st;
        if ((st = dev_alloc(b, &pp, (size_t)n * b->pp * kPairFields))) return st;
        if ((st = dev_alloc(b, &Qn, n))) return st;
        if ((st = launch_permute_pairs(b, c, d_perm, pairs, pao, pp, Qn))) return st;
        KS_HIP(hipStreamSynchronize(b->stream));
        b->d_pairs[c] = pairs;
        b->d_pair_ao[c] = pao;
        b->d_pp[c] = pp;
        b->d_Q[c] = Qn;
    }
    b->pairs_sorted = true;
    return KS_OK;
}

static void free_batch(ks_batch* b)
{
    if (!b) return;
    if (b->aux) (void)hipStreamSynchronize(b->aux);
    resolve_timers(b);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    else (void)hipDeviceSynchronize();
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    for (void* p : b->allocs) (void)hipFree(p);
    if (b->ev_grid) (void)hipEventDestroy(b->ev_grid);
    if (b->ev_main) (void)hipEventDestroy(b->ev_main);
    if (b->aux) (void)hipStreamDestroy(b->aux);
    if (b->h_nactive) (void)hipHostFree(b->h_nactive);
    delete b;
}

extern "C" {

void ks_default_options(ks_options* o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->xc = KS_XC_B3LYP;
    o->prec = KS_FP64;
    o->n_rad = 50;
    o->n_theta = 12;
    o->n_phi = 24;
    o->e_tol = 1e-9;
    o->comm_tol = 1e-7;
    o->max_iter = 100;
    o->diis_space = 8;
    o->jk_chunks = 0;
    o->xc_chunks = 0;
    o->guess = KS_GUESS_ATOM;
    o->xc_points = 0;
    o->xc_waves = 0;
}

const char* ks_last_error(void) { return g_err; }

static ks_status create_impl(const ks_options* opt, int n_mol, const int* n_atoms, const int* Z, const double* xyz,
                             const int* charge, void* stream, ks_batch* b);

ks_status ks_batch_create(const ks_options* opt, int n_mol, const int* n_atoms, const int* Z,
                          const double* xyz_angstrom, const int* charge, void* stream, ks_batch** out)
{
    g_err[0] = 0;
    if (!out) {
        set_error("out is NULL");
        return KS_EINVAL;
    }
    *out = nullptr;
    ks_batch* b = new (std::nothrow) ks_batch();
    if (!b) {
        set_error("host allocation failed");
        return KS_ENOMEM;
    }
    ks_status st = create_impl(opt, n_mol, n_atoms, Z, xyz_angstrom, charge, stream, b);
    if (st != KS_OK) {
        free_batch(b);
        return st;
    }
    *out = b;
    return KS_OK;
}

void ks_batch_destroy(ks_batch* b) { free_batch(b); }

}  // extern "C"

static ks_status create_impl(const ks_options* opt_in, int n_mol, const int* n_atoms, const int* Zin, const double* xyz,
                             const int* charge, void* stream, ks_batch* b)
{
    ks_options opt;
    ks_default_options(&opt);
    if (opt_in) opt = *opt_in;
    if (n_mol <= 0 || !n_atoms || !Zin || !xyz) {
        set_error("n_mol must be > 0 and n_atoms, Z, xyz non-NULL");
        return KS_EINVAL;
    }
    if (opt.xc < KS_XC_HF || opt.xc > KS_XC_B3LYP5 || (opt.prec != KS_FP64 && opt.prec != KS_MIXED)) {
        set_error("unknown xc or precision option");
        return KS_EINVAL;
    }
    for (int c = 0; c < kNClass; c++) {
        const int t = opt.eri_threads[c], u = opt.eri_unroll[c];
        if ((t != 0 && t != 64 && t != 128 && t != 256) || (u != 0 && u != 3 && u != 9)) {
            set_error("eri_threads must be 0, 64, 128 or 256 and eri_unroll 0, 3 or 9 (class %d: %d, %d)", c, t, u);
            return KS_EINVAL;
        }
    }
    if ((opt.direct != 0 && opt.direct != 1) || !(opt.schwarz_tol >= 0.0) || (opt.graphs != 0 && opt.graphs != 1)) {
        set_error("direct and graphs must be 0 or 1 and schwarz_tol >= 0");
        return KS_EINVAL;
    }
    if (opt.basis != KS_BASIS_STO3G && opt.basis != KS_BASIS_631G) {
        set_error("basis must be KS_BASIS_STO3G or KS_BASIS_631G");
        return KS_EINVAL;
    }
    if (opt.guess != KS_GUESS_ATOM && opt.guess != KS_GUESS_CORE) {
        set_error("unknown guess option %d", opt.guess);
        return KS_EINVAL;
    }
    if (opt.n_rad < 1 || opt.n_theta < 1 || opt.n_phi < 1 || opt.max_iter < 1 || opt.diis_space < 1 ||
        opt.diis_space > kMaxDiis || !(opt.e_tol > 0) || !(opt.comm_tol > 0)) {
        set_error("grid sizes, max_iter >= 1, 1 <= diis_space <= %d and positive tolerances required", kMaxDiis);
        return KS_EINVAL;
    }
    {
        const int cr = opt.coarse_rad, ct = opt.coarse_theta, cp = opt.coarse_phi;
        const bool off = cr == 0 && ct == 0 && cp == 0;
        if (!off && (cr < 1 || ct < 1 || cp < 1 || cr > opt.n_rad || ct > opt.n_theta || cp > opt.n_phi)) {
            set_error("coarse grid: all of coarse_rad, coarse_theta, coarse_phi 0 (off) or each in 1..the main grid's count");
            return KS_EINVAL;
        }
    }
    if (opt.prec == KS_MIXED) {
        opt.e_tol = std::max(opt.e_tol, kMixedETol);
        opt.comm_tol = std::max(opt.comm_tol, kMixedCommTol);
    }
    b->opt = opt;
    b->stream = (hipStream_t)stream;
    b->n_mol = n_mol;
    b->a0 = opt.xc == KS_XC_HF ? 1.0 : 0.20;
    const int maxn = opt.prec == KS_MIXED ? kMaxNbf : 82;
    b->pp = opt.basis == KS_BASIS_631G ? kPrimPairMax : kNPrimPair;

    long atom0 = 0, mat0 = 0, grid0 = 0, ao0 = 0;
    long qoff[kNClass] = {0, 0, 0, 0, 0, 0};
    std::vector<Pair> pairs[3];
    std::vector<int2> aoinfo;
    std::vector<long> qprefix[kNClass];
    for (int c = 0; c < kNClass; c++) qprefix[c].push_back(0);
    const long per_atom = (long)opt.n_rad * opt.n_theta * opt.n_phi;
    b->mol.resize(n_mol);
    for (int m = 0; m < n_mol; m++) {
        MolDesc& md = b->mol[m];
        std::memset(&md, 0, sizeof(md));
        const int na = n_atoms[m];
        if (na <= 0) {
            set_error("molecule %d: n_atoms must be > 0", m);
            return KS_EINVAL;
        }
        int ne = -(charge ? charge[m] : 0), nbf = 0;
        md.natom = na;
        md.atom0 = (int)atom0;
        md.shell0 = (int)b->shells.size();
        for (int a = 0; a < na; a++) {
            const int z = Zin[atom0 + a];
            double z1, z2;
            if (!element_zetas(z, z1, z2) || (opt.basis == KS_BASIS_631G && z != 1 && g631_heavy(z) < 0)) {
                set_error("molecule %d atom %d: element Z=%d is not in %s", m, a, z,
                          opt.basis == KS_BASIS_631G ? "{H, C, N, O} (6-31G)" : "{H, C, N, O, F}");
                return KS_EINVAL;
            }
            double p[3];
            for (int k = 0; k < 3; k++) {
                const double v = xyz[3 * (atom0 + a) + k];
                if (!std::isfinite(v)) {
                    set_error("molecule %d atom %d: non-finite coordinate", m, a);
                    return KS_EINVAL;
                }
                p[k] = v / kBohrAng;
            }
            for (int c = 0; c < a; c++) {
                const double* q = &b->R[3 * (atom0 + c)];
                const double d = std::sqrt((p[0] - q[0]) * (p[0] - q[0]) + (p[1] - q[1]) * (p[1] - q[1]) + (p[2] - q[2]) * (p[2] - q[2]));
                if (d < 0.1) {
                    set_error("molecule %d: atoms %d and %d closer than 0.1 bohr", m, c, a);
                    return KS_EINVAL;
                }
            }
            b->Z.push_back(z);
            for (int k = 0; k < 3; k++) b->R.push_back(p[k]);
            ne += z;
            Shell s{};
            for (int k = 0; k < 3; k++) s.A[k] = p[k];
            s.atom = a;
            nbf += add_atom_shells(b->shells, s, z, opt.basis, nbf);
        }
        if (ne <= 0 || (ne & 1)) {
            set_error("molecule %d: %d electrons; the restricted method needs a positive even count", m, ne);
            return KS_EINVAL;
        }
        if (nbf > maxn) {
            set_error("molecule %d: %d basis functions exceeds the %d supported in this precision", m, nbf, maxn);
            return KS_EUNSUPPORTED;
        }
        md.nbf = nbf;
        md.nocc = ne / 2;
        if (md.nocc > nbf) {
            set_error("molecule %d: more occupied orbitals than basis functions", m);
            return KS_EINVAL;
        }
        md.nshell = (int)b->shells.size() - md.shell0;
        md.np = (nbf + 15) / 16 * 16;
        md.ao0 = (int)ao0;
        md.mat0 = mat0;
        md.grid0 = grid0;
        md.ngrid = (long)na * per_atom;
        double enuc = 0.0;
        for (int a = 0; a < na; a++)
            for (int c = 0; c < a; c++) {
                const double* p = &b->R[3 * (atom0 + a)];
                const double* q = &b->R[3 * (atom0 + c)];
                enuc += Zin[atom0 + a] * Zin[atom0 + c] /
                        std::sqrt((p[0] - q[0]) * (p[0] - q[0]) + (p[1] - q[1]) * (p[1] - q[1]) + (p[2] - q[2]) * (p[2] - q[2]));
            }
        md.enuc = enuc;
        // AO table
        for (int s = md.shell0; s < md.shell0 + md.nshell; s++)
            for (int c = 0; c < (b->shells[s].L ? 3 : 1); c++) aoinfo.push_back(make_int2(s, c));
        // shell pairs by class (the p shell first in ps pairs)
        for (int c = 0; c < 3; c++) md.pair0[c] = (int)pairs[c].size();
        for (int sa = md.shell0; sa < md.shell0 + md.nshell; sa++)
            for (int sb = md.shell0; sb <= sa; sb++) {
                const int la = b->shells[sa].L, lb = b->shells[sb].L;
                if (la + lb == 1) pairs[1].push_back(la ? Pair{sa, sb} : Pair{sb, sa});
                else pairs[la + lb].push_back(Pair{sa, sb});
            }
        // anti-diagonal order (sa + sb, then sa): neighbouring pairs differ in
        // both shells, so lanes digesting neighbouring quartets scatter to
        // different J/K rows and columns
        for (int c = 0; c < 3; c++)
            std::stable_sort(pairs[c].begin() + md.pair0[c], pairs[c].end(), [](const Pair& x, const Pair& y) {
                return x.sa + x.sb != y.sa + y.sb ? x.sa + x.sb < y.sa + y.sb : x.sa < y.sa;
            });
        for (int c = 0; c < 3; c++) md.npair[c] = (int)pairs[c].size() - md.pair0[c];
        for (int c = 0; c < kNClass; c++) {
            const long nb = md.npair[class_bra(c)], nk = md.npair[class_ket(c)];
            md.nq[c] = class_tri(c) ? nb * (nb + 1) / 2 : nb * nk;
            md.q0[c] = qoff[c];
            qoff[c] += md.nq[c];
            qprefix[c].push_back(qoff[c]);
            b->nprimq += md.nq[c] * (long)b->pp * b->pp;
        }
        atom0 += na;
        mat0 += (long)nbf * nbf;
        grid0 += md.ngrid;
        ao0 += nbf;
        b->max_np = std::max(b->max_np, md.np);
        b->max_nshell = std::max(b->max_nshell, md.nshell);
    }
    b->nmat = mat0;
    b->ngrid = grid0;
    // the coarse start grids follow the main grids in the batch grid array
    b->coarse = opt.xc != KS_XC_HF && opt.coarse_rad > 0;
    if (b->coarse) {
        const long per_atom_c = (long)opt.coarse_rad * opt.coarse_theta * opt.coarse_phi;
        long gc = grid0;
        for (auto& md : b->mol) {
            md.gridc0 = gc;
            md.ngridc = (long)md.natom * per_atom_c;
            gc += md.ngridc;
        }
        b->ngridc = gc - grid0;
    }
    for (int c = 0; c < 3; c++) b->npairs[c] = (long)pairs[c].size();
    for (int c = 0; c < kNClass; c++) b->nq[c] = qoff[c];

    // work items
    // default: ~2048 J/K work groups per launch (8 per molecule at 256 molecules)
    const int jk_chunks = opt.jk_chunks > 0 ? opt.jk_chunks : std::max(1, std::min(64, (2048 + n_mol - 1) / n_mol));
    for (int m = 0; m < n_mol; m++)
        for (int c = 0; c < jk_chunks; c++) b->jk_items.push_back(JkItem{m, c, jk_chunks, 0});
    const int bp = xc_block_points(b);
    std::vector<int> xc_first;
    for (int m = 0; m < n_mol; m++) {
        xc_first.push_back((int)b->xc_items.size());
        const MolDesc& md = b->mol[m];
        // default: ~4096 work groups per launch (16 per molecule at 256
        // molecules), at most 64 per molecule
        long nch = opt.xc_chunks > 0 ? opt.xc_chunks : std::max(1, std::min(64, (4096 + n_mol - 1) / n_mol));
        nch = std::max(1L, std::min(nch, md.ngrid / (4L * bp)));
        for (long c = 0; c < nch; c++) {
            XcItem it{};
            it.mol = m;
            it.g0 = md.ngrid * c / nch;
            it.g1 = md.ngrid * (c + 1) / nch;
            b->xc_items.push_back(it);
        }
    }
    xc_first.push_back((int)b->xc_items.size());
    std::vector<int> xc_first_c;
    if (b->coarse) {
        for (int m = 0; m < n_mol; m++) {
            xc_first_c.push_back((int)b->xc_items.size());
            const MolDesc& md = b->mol[m];
            const long nfull = xc_first[m + 1] - xc_first[m];
            const long nch = std::max(1L, std::min(nfull, md.ngridc / (4L * bp)));
            for (long c = 0; c < nch; c++) {
                XcItem it{};
                it.mol = m;
                it.stage = 1;
                it.g0 = md.gridc0 - md.grid0 + md.ngridc * c / nch;
                it.g1 = md.gridc0 - md.grid0 + md.ngridc * (c + 1) / nch;
                b->xc_items.push_back(it);
            }
        }
        xc_first_c.push_back((int)b->xc_items.size());
    }

    // device memory
    ks_status st;
    std::vector<double> tab, rad, ang, Zc(b->Z.begin(), b->Z.end());
    build_boys_table(tab);
    std::vector<float> tabf(tab.begin(), tab.end());
    std::vector<double> boys_rows;
    build_boys_rows(boys_rows);
    radial_rule(opt.n_rad, rad);
    gauss_legendre(opt.n_theta, ang);
    std::vector<long> ptoff;
    long pt = 0;
    for (auto& md : b->mol) {
        ptoff.push_back(pt);
        pt += (long)md.np * md.np;
    }
    b->npt_total = pt;
    KS_HIP(hipStreamCreateWithFlags(&b->aux, hipStreamNonBlocking));
    KS_HIP(hipEventCreateWithFlags(&b->ev_main, hipEventDisableTiming));
    KS_HIP(hipEventCreateWithFlags(&b->ev_grid, hipEventDisableTiming));
    if ((st = upload(b, &b->d_mol, b->mol))) return st;
    if ((st = upload(b, &b->d_shells, b->shells))) return st;
    if ((st = upload(b, &b->d_aoinfo, aoinfo))) return st;
    if ((st = upload(b, &b->d_R, b->R))) return st;
    if ((st = upload(b, &b->d_Zc, Zc))) return st;
    if ((st = upload(b, &b->d_boys, tab))) return st;
    if ((st = upload(b, &b->d_boys_f, tabf))) return st;
    if ((st = upload(b, &b->d_boys_rows, boys_rows))) return st;
    if ((st = upload(b, &b->d_radial, rad))) return st;
    if ((st = upload(b, &b->d_ang, ang))) return st;
    if (b->coarse) {
        std::vector<double> radc, angc;
        radial_rule(opt.coarse_rad, radc);
        gauss_legendre(opt.coarse_theta, angc);
        if ((st = upload(b, &b->d_radial_c, radc))) return st;
        if ((st = upload(b, &b->d_ang_c, angc))) return st;
        if ((st = upload(b, &b->d_xc_first_c, xc_first_c))) return st;
    }
    if ((st = upload(b, &b->d_ptoff, ptoff))) return st;
    if ((st = upload(b, &b->d_jk_items, b->jk_items))) return st;
    if ((st = upload(b, &b->d_xc_items, b->xc_items))) return st;
    if ((st = upload(b, &b->d_xc_first, xc_first))) return st;
    for (int c = 0; c < 3; c++) {
        std::vector<int2> pao(pairs[c].size());
        for (size_t i = 0; i < pairs[c].size(); i++) {
            const Pair& pr = pairs[c][i];
            pao[i] = make_int2(b->shells[pr.sa].ao | (pr.sa == pr.sb ? 1 << 16 : 0), b->shells[pr.sb].ao);
        }
        if ((st = upload(b, &b->d_pair_ao[c], pao))) return st;
        if ((st = upload(b, &b->d_pairs[c], pairs[c]))) return st;
        if ((st = dev_alloc(b, &b->d_pp[c], pairs[c].size() * (size_t)b->pp * kPairFields))) return st;
        if ((st = dev_alloc(b, &b->d_Q[c], pairs[c].size()))) return st;
    }
    for (int c = 0; c < kNClass; c++)
        if ((st = upload(b, &b->d_qoff[c], qprefix[c]))) return st;
    std::vector<MolState> s0(n_mol);
    std::memset(s0.data(), 0, sizeof(MolState) * n_mol);
    for (auto& x : s0) {
        x.stage = b->coarse ? 1 : 0;
        x.it_full = 1;
    }
    if ((st = upload(b, &b->d_state, s0))) return st;
    double** mats[] = {&b->d_S, &b->d_T, &b->d_V, &b->d_H, &b->d_X, &b->d_F, &b->d_P,
                       &b->d_J, &b->d_K, &b->d_Vxc, &b->d_Fp, &b->d_C, &b->d_Pprev, &b->d_Cp};
    for (double** p : mats)
        if ((st = dev_alloc(b, p, (size_t)b->nmat))) return st;
    if ((st = dev_alloc(b, &b->d_eps, (size_t)ao0))) return st;
    if ((st = dev_alloc(b, &b->d_work, 3 * (size_t)b->nmat))) return st;
    if ((st = dev_alloc(b, &b->d_Fh, (size_t)opt.diis_space * b->nmat))) return st;
    if ((st = dev_alloc(b, &b->d_Eh, (size_t)opt.diis_space * b->nmat))) return st;
    const size_t es = opt.prec == KS_MIXED ? sizeof(float) : sizeof(double);
    const size_t np2 = (size_t)b->max_np * b->max_np;
    unsigned char* tmp;
    if ((st = dev_alloc(b, &tmp, es * (size_t)pt))) return st;
    b->d_Pt = tmp;
    if ((st = dev_alloc(b, &tmp, sizeof(double) * 2 * np2 * b->jk_items.size()))) return st;
    b->d_jk_part = tmp;
    if ((st = dev_alloc(b, &tmp, es * np2 * b->xc_items.size()))) return st;
    b->d_xc_part = tmp;
    if ((st = dev_alloc(b, &b->d_xc_exc, b->xc_items.size()))) return st;
    if ((st = dev_alloc(b, &b->d_exc, (size_t)n_mol))) return st;
    if ((st = dev_alloc(b, &b->d_nactive, 1))) return st;
    if ((st = dev_alloc(b, &b->d_eterms, 6 * (size_t)n_mol))) return st;
    if ((st = dev_alloc(b, &b->d_have_warm, (size_t)n_mol))) return st;
    KS_HIP(hipHostMalloc((void**)&b->h_nactive, sizeof(int), hipHostMallocDefault));
    KS_HIP(hipMemsetAsync(b->d_Vxc, 0, sizeof(double) * b->nmat, b->stream));
    KS_HIP(hipMemsetAsync(b->d_J, 0, sizeof(double) * b->nmat, b->stream));
    KS_HIP(hipMemsetAsync(b->d_K, 0, sizeof(double) * b->nmat, b->stream));
    KS_HIP(hipMemsetAsync(b->d_Pprev, 0, sizeof(double) * b->nmat, b->stream));
    KS_HIP(hipMemsetAsync(b->d_exc, 0, sizeof(double) * n_mol, b->stream));
    KS_HIP(hipMemsetAsync(b->d_have_warm, 0, sizeof(int) * n_mol, b->stream));
    KS_HIP(hipStreamSynchronize(b->stream));
    return KS_OK;
}

// ---------------------------------------------------------------------------
// entry points
// ---------------------------------------------------------------------------
#define CHECK_B(b)                             \
    do {                                       \
        g_err[0] = 0;                          \
        if (!(b)) {                            \
            set_error("batch handle is NULL"); \
            return KS_EINVAL;                  \
        }                                      \
    } while (0)

extern "C" {

ks_status ks_batch_sizes(const ks_batch* b, int mol, int* nbf, int* nocc, long* n_eri, long* n_grid)
{
    CHECK_B(b);
    if (mol < 0 || mol >= b->n_mol) {
        set_error("molecule index %d out of range", mol);
        return KS_EINVAL;
    }
    const MolDesc& md = b->mol[mol];
    const long np = (long)md.nbf * (md.nbf + 1) / 2;
    if (nbf) *nbf = md.nbf;
    if (nocc) *nocc = md.nocc;
    if (n_eri) *n_eri = np * (np + 1) / 2;
    if (n_grid) *n_grid = md.ngrid;
    return KS_OK;
}

ks_status ks_batch_quartets(const ks_batch* b, long* nq, long* nprim)
{
    CHECK_B(b);
    long t = 0;
    for (int c = 0; c < kNClass; c++) t += b->nq[c];
    if (nq) *nq = t;
    if (nprim) *nprim = b->nprimq;
    return KS_OK;
}

ks_status ks_setup(ks_batch* b)
{
    CHECK_B(b);
    if (b->setup_done) return KS_OK;
    ks_status st;
    if ((st = launch_pairs(b))) return st;
    if ((st = launch_int1e(b))) return st;
    if ((st = launch_lowdin(b))) return st;
    std::vector<MolState> s(b->n_mol);
    KS_HIP(hipMemcpyAsync(s.data(), b->d_state, sizeof(MolState) * b->n_mol, hipMemcpyDeviceToHost, b->stream));
    KS_HIP(hipStreamSynchronize(b->stream));
    for (int m = 0; m < b->n_mol; m++)
        if (s[m].status == -1) {
            set_error("molecule %d: near-singular overlap (smallest eigenvalue < 1e-8)", m);
            return KS_EINVAL;
        }
    if (b->opt.xc != KS_XC_HF) {
        if ((st = dev_alloc(b, &b->d_grid, 4 * (size_t)(b->ngrid + b->ngridc)))) return st;
        KS_HIP(hipEventRecord(b->ev_main, b->stream));
        KS_HIP(hipStreamWaitEvent(b->aux, b->ev_main, 0));
        if ((st = launch_grid(b, b->aux))) return st;
        KS_HIP(hipEventRecord(b->ev_grid, b->aux));
        b->grid_pending = true;
    }
    if ((st = launch_guess(b))) return st;
    b->setup_done = true;
    b->guess_done = true;
    return KS_OK;
}

ks_status eri_build(ks_batch* b)
{
    CHECK_B(b);
    if (b->eri_done) return KS_OK;
    ks_status st;
    if (!b->setup_done && (st = ks_setup(b))) return st;
    if (b->opt.direct || b->opt.schwarz_tol > 0.0) {
        if ((st = launch_schwarz(b))) return st;
    }
    if (b->opt.direct) {        // integral-direct: nothing is stored
        if ((st = sort_pairs_by_schwarz(b))) return st;
        b->eri_done = true;
        return KS_OK;
    }
    const size_t es = b->opt.prec == KS_MIXED ? sizeof(float) : sizeof(double);
    for (int c = 0; c < kNClass; c++) {
        unsigned char* p;
        if ((st = dev_alloc(b, &p, es * (size_t)b->nq[c] * class_ncomp(c)))) return st;
        b->d_eri[c] = p;
    }
    if ((st = launch_eri(b))) return st;
    b->eri_done = true;
    return KS_OK;
}

ks_status jk_build(ks_batch* b, const void* P, void* J, void* K)
{
    CHECK_B(b);
    if (!P || !J || !K) {
        set_error("P, J and K must be device pointers");
        return KS_EINVAL;
    }
    if (!b->eri_done) {
        set_error("jk_build before eri_build");
        return KS_ESTATE;
    }
    ks_status st = launch_jk(b, (const double*)P, (double*)J, (double*)K, false, false, false);
    if (st) return st;
    KS_HIP(hipStreamSynchronize(b->stream));
    return KS_OK;
}

ks_status xc_build(ks_batch* b, const void* P, void* V, double* Exc)
{
    CHECK_B(b);
    if (!P || !V) {
        set_error("P and Vxc must be device pointers");
        return KS_EINVAL;
    }
    ks_status st;
    if (!b->setup_done && (st = ks_setup(b))) return st;
    if (b->opt.xc == KS_XC_HF) {
        KS_HIP(hipMemsetAsync(V, 0, sizeof(double) * b->nmat, b->stream));
        KS_HIP(hipStreamSynchronize(b->stream));
        if (Exc)
            for (int m = 0; m < b->n_mol; m++) Exc[m] = 0.0;
        return KS_OK;
    }
    if ((st = launch_xc(b, (const double*)P, (double*)V, false))) return st;
    if (Exc) KS_HIP(hipMemcpyAsync(Exc, b->d_exc, sizeof(double) * b->n_mol, hipMemcpyDeviceToHost, b->stream));
    KS_HIP(hipStreamSynchronize(b->stream));
    return KS_OK;
}

ks_status fock_build(ks_batch* b, const void* Pin, void* F, double* E_terms)
{
    CHECK_B(b);
    ks_status st;
    if (!b->eri_done && (st = eri_build(b))) return st;
    const double* P = Pin ? (const double*)Pin : b->d_P;
    if ((st = launch_jk(b, P, b->d_J, b->d_K, false, false, true))) return st;
    if (b->opt.xc != KS_XC_HF) {
        if ((st = launch_xc(b, P, b->d_Vxc, false))) return st;
    }
    double* Fo = F ? (double*)F : b->d_work;
    if ((st = launch_fock(b, P, b->d_J, b->d_K, b->d_Vxc, Fo, false, b->d_eterms))) return st;
    if (E_terms)
        KS_HIP(hipMemcpyAsync(E_terms, b->d_eterms, sizeof(double) * 6 * b->n_mol, hipMemcpyDeviceToHost, b->stream));
    KS_HIP(hipStreamSynchronize(b->stream));
    return KS_OK;
}

}  // extern "C"

namespace ks {

ks_status grid_wait(ks_batch* b)
{
    if (b->grid_pending) {
        KS_HIP(hipStreamWaitEvent(b->stream, b->ev_grid, 0));
        b->grid_pending = false;
    }
    return KS_OK;
}

}  // namespace ks

namespace ks {

// The launches of one SCF iteration (every iteration issues the same ones
// with the same arguments; the kernels skip retired molecules).
static ks_status enqueue_iteration(ks_batch* b)
{
    ks_status st;
    // mixed and integral-direct paths: incremental J/K from P - Pprev
    const bool inc = b->opt.prec == KS_MIXED || b->opt.direct;
    if ((st = launch_jk(b, b->d_P, b->d_J, b->d_K, true, inc, true))) return st;
    if (b->opt.xc != KS_XC_HF && (st = launch_xc(b, b->d_P, b->d_Vxc, true))) return st;
    if ((st = launch_fock(b, b->d_P, b->d_J, b->d_K, b->d_Vxc, b->d_F, true, nullptr))) return st;
    if ((st = launch_iteration_tail(b))) return st;
    if ((st = launch_count_active(b))) return st;
    KS_HIP(hipMemcpyAsync(b->h_nactive, b->d_nactive, sizeof(int), hipMemcpyDeviceToHost, b->stream));
    return KS_OK;
}

// One SCF iteration queued on the batch stream, without waiting: the count of
// still-active molecules lands in pinned host memory (read by step_finish).
// With options.graphs the second iteration is captured into a graph (the
// first one also waits for the grid and may build the Schwarz order) and
// every later one replays it.
ks_status step_launch(ks_batch* b)
{
    ks_status st;
    if (!b->eri_done && (st = eri_build(b))) return st;
    const bool graph = b->opt.graphs && b->stream && !b->timing && b->iter >= 1 && !b->grid_pending;
    if (graph && b->gexec) {
        KS_HIP(hipGraphLaunch(b->gexec, b->stream));
        b->iter++;
        return KS_OK;
    }
    if (!graph) {
        if ((st = enqueue_iteration(b))) return st;
        b->iter++;
        return KS_OK;
    }
    KS_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    st = enqueue_iteration(b);
    hipGraph_t gr = nullptr;
    const hipError_t e = hipStreamEndCapture(b->stream, &gr);
    if (!st && e != hipSuccess) {
        set_error("graph capture of the SCF iteration failed: %s", hipGetErrorString(e));
        st = KS_EDEVICE;
    }
    if (!st) {
        const hipError_t ei = hipGraphInstantiate(&b->gexec, gr, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
            set_error("graph instantiation failed: %s", hipGetErrorString(ei));
            b->gexec = nullptr;
            st = KS_EDEVICE;
        }
    }
    if (gr) (void)hipGraphDestroy(gr);
    if (st) return st;
    KS_HIP(hipGraphLaunch(b->gexec, b->stream));
    b->iter++;
    return KS_OK;
}

ks_status step_finish(ks_batch* b, int* n_active)
{
    KS_HIP(hipStreamSynchronize(b->stream));
    if (n_active) *n_active = *b->h_nactive;
    return KS_OK;
}

size_t batch_device_bytes(const ks_batch* b) { return b->alloc_bytes; }

}  // namespace ks

extern "C" {

ks_status scf_step(ks_batch* b, int* n_active)
{
    CHECK_B(b);
    ks_status st = step_launch(b);
    if (st) return st;
    return step_finish(b, n_active);
}

ks_status scf_solve_many(ks_batch* const* bs, int n)
{
    if (!bs || n <= 0) {
        set_error("scf_solve_many: NULL batch list or n <= 0");
        return KS_EINVAL;
    }
    for (int i = 0; i < n; i++) {
        CHECK_B(bs[i]);
        for (int k = 0; k < i; k++)
            if (bs[k] == bs[i]) {
                set_error("scf_solve_many: batch %d appears twice", i);
                return KS_EINVAL;
            }
    }
    // each batch's next iteration is queued as soon as its previous one has
    // been read back, so the GPU always holds work of the other batches
    std::vector<char> active(n, 1);
    std::vector<int> steps(n, 0);
    ks_status st;
    for (int i = 0; i < n; i++) {
        if ((st = step_launch(bs[i]))) return st;
        steps[i] = 1;
    }
    for (int left = n; left > 0;) {
        for (int i = 0; i < n; i++) {
            if (!active[i]) continue;
            int na = 0;
            if ((st = step_finish(bs[i], &na))) return st;
            if (na == 0) {
                active[i] = 0;
                left--;
            } else if (steps[i] >= bs[i]->opt.max_iter + 2) {
                set_error("scf_solve_many: batch %d still active after max_iter + 2 steps", i);
                return KS_ESTATE;
            } else {
                if ((st = step_launch(bs[i]))) return st;
                steps[i]++;
            }
        }
    }
    return KS_OK;
}

ks_status scf_solve(ks_batch* b)
{
    CHECK_B(b);
    ks_status st;
    for (int it = 0; it <= b->opt.max_iter + 1; it++) {
        int na = 0;
        if ((st = scf_step(b, &na))) return st;
        if (na == 0) return KS_OK;
    }
    set_error("scf_solve: molecules still active after max_iter + 2 steps");
    return KS_ESTATE;
}

ks_status ks_get_result(const ks_batch* b, int mol, double* E, double* eps, double* P, double* homo, double* lumo,
                        double* gap, int* status, int* n_iter)
{
    CHECK_B(b);
    if (mol < 0 || mol >= b->n_mol) {
        set_error("molecule index %d out of range", mol);
        return KS_EINVAL;
    }
    const MolDesc& md = b->mol[mol];
    MolState s;
    std::vector<double> e(md.nbf);
    KS_HIP(hipMemcpyAsync(&s, b->d_state + mol, sizeof(MolState), hipMemcpyDeviceToHost, b->stream));
    KS_HIP(hipMemcpyAsync(e.data(), b->d_eps + md.ao0, sizeof(double) * md.nbf, hipMemcpyDeviceToHost, b->stream));
    if (P) KS_HIP(hipMemcpyAsync(P, b->d_P + md.mat0, sizeof(double) * md.nbf * md.nbf, hipMemcpyDeviceToHost, b->stream));
    KS_HIP(hipStreamSynchronize(b->stream));
    if (E) *E = s.E;
    if (eps) std::memcpy(eps, e.data(), sizeof(double) * md.nbf);
    const double h = e[md.nocc - 1], l = md.nocc < md.nbf ? e[md.nocc] : NAN;
    if (homo) *homo = h;
    if (lumo) *lumo = l;
    if (gap) *gap = l - h;
    if (status) *status = s.status;
    if (n_iter) *n_iter = s.iter;
    return KS_OK;
}

ks_status ks_get_eri(const ks_batch* b, int mol, double* out)
{
    CHECK_B(b);
    if (mol < 0 || mol >= b->n_mol || !out) {
        set_error("bad molecule index or NULL output");
        return KS_EINVAL;
    }
    if (!b->eri_done) {
        set_error("ks_get_eri before eri_build");
        return KS_ESTATE;
    }
    if (b->opt.direct) {
        set_error("ks_get_eri: an integral-direct batch stores no integrals");
        return KS_ESTATE;
    }
    long neri;
    ks_batch_sizes(b, mol, nullptr, nullptr, &neri, nullptr);
    double* d = nullptr;
    KS_HIP(hipMalloc(&d, sizeof(double) * neri));
    ks_status st = launch_eri_unpack(b, mol, d);
    if (st == KS_OK) {
        hipError_t e = hipMemcpyAsync(out, d, sizeof(double) * neri, hipMemcpyDeviceToHost, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        if (e != hipSuccess) {
            set_error("ks_get_eri copy failed: %s", hipGetErrorString(e));
            st = KS_EDEVICE;
        }
    }
    (void)hipFree(d);
    return st;
}

// Staging array of ks_get_eri_window (callers that cannot allocate device
// memory): a file-scope device array, so each device holds one copy for the
// life of the process.  In host code its name is not a device address: the
// address is looked up once per device (hipGetSymbolAddress, with that device
// current) and only that address is passed to kernels and copies.
static __device__ __align__(256) double scratch[KS_ERI_WINDOW_MAX];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {};

static ks_status scratch_address(double** out)
{
    int dev = -1;
    KS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device %d out of range for the staging array", dev);
        return KS_EDEVICE;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            set_error("hipGetSymbolAddress of the staging array failed: %s", hipGetErrorString(e));
            return KS_EDEVICE;
        }
        g_scratch_ptr[dev] = (double*)p;
    }
    *out = g_scratch_ptr[dev];
    return KS_OK;
}

ks_status ks_get_eri_window(const ks_batch* b, int mol, long lo, long count, double* out)
{
    CHECK_B(b);
    if (mol < 0 || mol >= b->n_mol || (!out && count > 0)) {
        set_error("bad molecule index or NULL output");
        return KS_EINVAL;
    }
    if (!b->eri_done) {
        set_error("ks_get_eri_window before eri_build");
        return KS_ESTATE;
    }
    if (b->opt.direct) {
        set_error("ks_get_eri_window: an integral-direct batch stores no integrals");
        return KS_ESTATE;
    }
    if (count < 0 || count > KS_ERI_WINDOW_MAX) {
        set_error("window of %ld integrals: at most %d per call", count, (int)KS_ERI_WINDOW_MAX);
        return KS_EINVAL;
    }
    long neri;
    ks_batch_sizes(b, mol, nullptr, nullptr, &neri, nullptr);
    if (lo < 0 || lo + count > neri) {
        set_error("window %ld .. %ld outside the %ld packed integrals of molecule %d", lo, lo + count, neri, mol);
        return KS_EINVAL;
    }
    if (count == 0) return KS_OK;
    double* d = nullptr;
    ks_status st = scratch_address(&d);
    if (st) return st;
    if ((st = launch_eri_unpack_window(b, mol, lo, lo + count, d))) return st;
    KS_HIP(hipMemcpyAsync(out, d, sizeof(double) * count, hipMemcpyDeviceToHost, b->stream));
    KS_HIP(hipStreamSynchronize(b->stream));
    return KS_OK;
}

ks_status ks_get_matrix(const ks_batch* b, int mol, int which, double* out)
{
    CHECK_B(b);
    if (mol < 0 || mol >= b->n_mol || !out) {
        set_error("bad molecule index or NULL output");
        return KS_EINVAL;
    }
    const double* src[] = {b->d_S, b->d_T, b->d_V, b->d_X, b->d_F, b->d_P, b->d_J, b->d_K, b->d_Vxc};
    if (which < 0 || which > 8) {
        set_error("matrix selector %d out of range", which);
        return KS_EINVAL;
    }
    const MolDesc& md = b->mol[mol];
    KS_HIP(hipMemcpyAsync(out, src[which] + md.mat0, sizeof(double) * md.nbf * md.nbf, hipMemcpyDeviceToHost, b->stream));
    KS_HIP(hipStreamSynchronize(b->stream));
    return KS_OK;
}

ks_status ks_get_grid(const ks_batch* b, int mol, double* out)
{
    CHECK_B(b);
    if (mol < 0 || mol >= b->n_mol || !out) {
        set_error("bad molecule index or NULL output");
        return KS_EINVAL;
    }
    if (!b->d_grid) {
        set_error("no grid (Hartree-Fock batch or ks_setup not called)");
        return KS_ESTATE;
    }
    const MolDesc& md = b->mol[mol];
    ks_status st = grid_wait(const_cast<ks_batch*>(b));
    if (st) return st;
    KS_HIP(hipMemcpyAsync(out, b->d_grid + 4 * md.grid0, sizeof(double) * 4 * md.ngrid, hipMemcpyDeviceToHost, b->stream));
    KS_HIP(hipStreamSynchronize(b->stream));
    return KS_OK;
}

void ks_set_timing(ks_batch* b, int on)
{
    if (!b) return;
    resolve_timers(b);
    b->timing = on != 0;
    b->tnames.clear();
    b->tms.clear();
}

int ks_kernel_times(const ks_batch* b, const char** names, double* ms, int cap)
{
    if (!b) return 0;
    ks_batch* bb = const_cast<ks_batch*>(b);
    resolve_timers(bb);
    int n = (int)b->tnames.size();
    for (int i = 0; i < n && i < cap; i++) {
        names[i] = b->tnames[i].c_str();
        ms[i] = b->tms[2 * i] / std::max(1.0, b->tms[2 * i + 1]);
    }
    return n;
}

int ks_kernel_counts(const ks_batch* b, double* launches, int cap)
{
    if (!b) return 0;
    resolve_timers(const_cast<ks_batch*>(b));
    int n = (int)b->tnames.size();
    for (int i = 0; i < n && i < cap; i++) launches[i] = b->tms[2 * i + 1];
    return n;
}

ks_status ks_get_convergence(const ks_batch* b, int mol, double* E, double* dE, double* err)
{
    CHECK_B(b);
    if (mol < 0 || mol >= b->n_mol) {
        set_error("molecule index %d out of range", mol);
        return KS_EINVAL;
    }
    MolState s;
    KS_HIP(hipMemcpyAsync(&s, b->d_state + mol, sizeof(MolState), hipMemcpyDeviceToHost, b->stream));
    KS_HIP(hipStreamSynchronize(b->stream));
    if (E) *E = s.E;
    if (dE) *dE = s.dE;
    if (err) *err = s.err;
    return KS_OK;
}

ks_status ks_get_results(const ks_batch* b, double* E, double* homo, double* lumo, double* gap, int* status,
                         int* n_iter, int* n_coarse, double* eps, double* P)
{
    CHECK_B(b);
    const int n = b->n_mol;
    long nao = 0;
    for (const MolDesc& md : b->mol) nao += md.nbf;
    std::vector<MolState> s(n);
    std::vector<double> e(nao);
    KS_HIP(hipMemcpyAsync(s.data(), b->d_state, sizeof(MolState) * n, hipMemcpyDeviceToHost, b->stream));
    KS_HIP(hipMemcpyAsync(e.data(), b->d_eps, sizeof(double) * nao, hipMemcpyDeviceToHost, b->stream));
    // the N x N blocks are contiguous in molecule order (mat0 = sum of nbf^2 before)
    if (P) KS_HIP(hipMemcpyAsync(P, b->d_P, sizeof(double) * b->nmat, hipMemcpyDeviceToHost, b->stream));
    KS_HIP(hipStreamSynchronize(b->stream));
    if (eps) std::memcpy(eps, e.data(), sizeof(double) * nao);
    for (int m = 0; m < n; m++) {
        const MolDesc& md = b->mol[m];
        const double h = e[md.ao0 + md.nocc - 1], l = md.nocc < md.nbf ? e[md.ao0 + md.nocc] : NAN;
        if (E) E[m] = s[m].E;
        if (homo) homo[m] = h;
        if (lumo) lumo[m] = l;
        if (gap) gap[m] = l - h;
        if (status) status[m] = s[m].status;
        if (n_iter) n_iter[m] = s[m].iter;
        if (n_coarse) n_coarse[m] = s[m].stage ? s[m].iter : s[m].it_full - 1;
    }
    return KS_OK;
}

ks_status ks_get_iterations(const ks_batch* b, int mol, int* n_iter, int* n_coarse)
{
    CHECK_B(b);
    if (mol < 0 || mol >= b->n_mol) {
        set_error("molecule index %d out of range", mol);
        return KS_EINVAL;
    }
    MolState s;
    KS_HIP(hipMemcpyAsync(&s, b->d_state + mol, sizeof(MolState), hipMemcpyDeviceToHost, b->stream));
    KS_HIP(hipStreamSynchronize(b->stream));
    if (n_iter) *n_iter = s.iter;
    if (n_coarse) *n_coarse = s.stage ? s.iter : s.it_full - 1;
    return KS_OK;
}

}  // extern "C"
