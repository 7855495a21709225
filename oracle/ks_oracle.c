/*
 * ks_oracle.c -- plain, slow FP64 CPU oracle for the restricted Kohn-Sham
 * (B3LYP / STO-3G) SCF of arxiv 2311.01135 ("Generating QM1B with PySCF_IPU").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or generator with the HIP path.
 *
 * What it computes (paper section 3.1, equation "roothaan" and the lines
 * under it): the Roothaan-Hall fixed point [V+T+J(rho)+K(rho)+V_XC(rho)] C =
 * S C eps with rho = C D C^T (D = 2 on the occupied orbitals),
 * J_kl = sum_ij I_ijkl rho_ij and K_il = -1/2 sum_jk I_ijkl rho_jk; the
 * B3LYP exact-exchange fraction a0 scales that K (the paper does not print
 * a0; we take 0.20).  Iteration 0 precomputes V, T, S and the ERIs, then
 * every iteration forms rho, V_XC, J, K and solves the generalised eigen-
 * problem (same passage).  The HL gap is reported as eps_LUMO - eps_HOMO
 * (positive; the paper prints the other sign).
 *
 * Textbook pieces the paper cites but does not print:
 *   STO-3G (Hehre, Stewart, Pople 1969): universal zeta=1 expansions scaled
 *     by zeta^2;
 *   6-31G (Hehre, Ditchfield, Pople 1972; H from the 31G set), H, C, N, O:
 *     a six-primitive core s shell and a 3 + 1 split valence (sp shells
 *     sharing exponents);
 *   Obara-Saika recurrences (J. Chem. Phys. 84, 3963 (1986)) for S, T, V
 *     and the ERIs (vertical recurrence + horizontal transfer);
 *   Boys function: F0 = 1/2 sqrt(pi/T) erf(sqrt T); F_m by series + downward
 *     recursion for T < 30 and upward recursion above;
 *   Treutler-Ahlrichs M4 radial grid (xi = 1, Chebyshev 2nd kind nodes),
 *     Gauss-Legendre x trapezoid angular grid, Becke fuzzy cells (3 steps,
 *     no size adjustment);
 *   B3LYP = 0.08 Slater + 0.72 B88 + 0.19 VWN + 0.81 LYP + 0.20 HF exchange,
 *     VWN in the RPA fit (default) or VWN5; closed-shell LYP in the
 *     gradient-only form; points with rho < 1e-12 are skipped;
 *   Loewdin S^-1/2, core-Hamiltonian guess, DIIS (Pulay) on the
 *     orthogonalised commutator, cyclic Jacobi eigensolver.
 *
 * Parity status: every function here is pinned by the CPU tests (closed
 * forms, brute force, textbook H2 values); the full B3LYP SCF energy of a
 * generated molecule has no external value and is pinned only through its
 * components ("parity unpinned" for that end-to-end number).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846
#define ORC_BOHR_ANG 0.52917721092

/* ------------------------------------------------------------------ */
/* STO-3G (Hehre, Stewart, Pople 1969): zeta = 1 expansions            */
/* ------------------------------------------------------------------ */
static const double STO1S_A[3] = {2.227660584, 0.4057711562, 0.1098175104};
static const double STO1S_D[3] = {0.1543289673, 0.5353281423, 0.4446345422};
static const double STO2SP_A[3] = {0.9942027, 0.2310313, 0.0751386};
static const double STO2S_D[3] = {-0.09996723, 0.39951283, 0.70011547};
static const double STO2P_D[3] = {0.15591627, 0.60768372, 0.39195739};

/* ------------------------------------------------------------------ */
/* 6-31G: per element the core 1s (6), inner valence sp (3) and outer  */
/* valence sp (1) shells; H: 31G (3 + 1).  Exponents, s and p          */
/* contraction coefficients.                                           */
/* ------------------------------------------------------------------ */
typedef struct { double a[6], d[6]; } g1s_t;
typedef struct { double a[3], ds[3], dp[3]; double a3; } gsp_t;
static const g1s_t G631_1S[3] = {   /* C, N, O */
    {{3047.5249, 457.36951, 103.94869, 29.210155, 9.2866630, 3.1639270},
     {0.0018347, 0.0140373, 0.0688426, 0.2321844, 0.4679413, 0.3623120}},
    {{4173.5110, 627.45790, 142.90210, 40.234330, 12.820210, 4.3904370},
     {0.0018348, 0.0139950, 0.0685870, 0.2322410, 0.4690700, 0.3604550}},
    {{5484.6717, 825.23495, 188.04696, 52.964500, 16.897570, 5.7996353},
     {0.0018311, 0.0139501, 0.0684451, 0.2327143, 0.4701930, 0.3585209}}};
static const gsp_t G631_SP[3] = {
    {{7.8682724, 1.8812885, 0.5442493}, {-0.1193324, -0.1608542, 1.1434564}, {0.0689991, 0.3164240, 0.7443083},
     0.1687144},
    {{11.626358, 2.7162800, 0.7722180}, {-0.1149610, -0.1691180, 1.1458520}, {0.0675800, 0.3239070, 0.7408950},
     0.2120313},
    {{15.539616, 3.5999336, 1.0137618}, {-0.1107775, -0.1480263, 1.1307670}, {0.0708743, 0.3397528, 0.7271586},
     0.2700058}};
static const double G631_H_A[3] = {18.7311370, 2.8253937, 0.6401217};
static const double G631_H_D[3] = {0.03349460, 0.23472695, 0.81375733};
static const double G631_H_A2 = 0.1612778;

static int zeta_of(int Z, double *z1, double *z2)
{
    switch (Z) {
    case 1: *z1 = 1.24; *z2 = 0.0; return 1;
    case 6: *z1 = 5.67; *z2 = 1.72; return 1;
    case 7: *z1 = 6.67; *z2 = 1.95; return 1;
    case 8: *z1 = 7.66; *z2 = 2.25; return 1;
    case 9: *z1 = 8.65; *z2 = 2.55; return 1;
    default: return 0;
    }
}

typedef struct {
    int L;          /* 0 or 1 */
    int atom;
    int bf0;        /* first AO index */
    int np;         /* primitives */
    double A[3];
    double a[6];
    double c[6];    /* contraction coefficient x primitive norm x renorm */
    double occ;     /* initial-guess occupation per function of the shell */
} oshell;

typedef struct {
    int natom, nshell, nbf, nelec, nocc;
    int *Z;
    double *R;      /* bohr, [natom][3] */
    oshell *sh;
    int *bf_shell;  /* AO -> shell */
    int *bf_comp;   /* AO -> Cartesian component (0 = s, 1..3 = x,y,z) */
} omol;

/* ------------------------------------------------------------------ */
/* Boys function F_m(T) = int_0^1 t^{2m} exp(-T t^2) dt                */
/* ------------------------------------------------------------------ */
void orc_boys(int mmax, double T, double *F)
{
    int m;
    if (T < 30.0) {
        /* series for F_mmax, then downward recursion */
        double term = 1.0 / (2 * mmax + 1), sum = term, eT = exp(-T);
        int k;
        for (k = 1; k < 200; k++) {
            term *= 2.0 * T / (2 * mmax + 2 * k + 1);
            sum += term;
            if (term < 1e-17 * sum) break;
        }
        F[mmax] = eT * sum;
        for (m = mmax - 1; m >= 0; m--) F[m] = (2.0 * T * F[m + 1] + eT) / (2 * m + 1);
        if (T > 0.0) F[0] = 0.5 * sqrt(ORC_PI / T) * erf(sqrt(T));
    } else {
        double eT = exp(-T);
        F[0] = 0.5 * sqrt(ORC_PI / T) * erf(sqrt(T));
        for (m = 0; m < mmax; m++) F[m + 1] = ((2 * m + 1) * F[m] - eT) / (2.0 * T);
    }
}

/* ------------------------------------------------------------------ */
/* molecule + basis                                                    */
/* ------------------------------------------------------------------ */
static double prim_norm(int L, double a)
{
    double n = pow(2.0 * a / ORC_PI, 0.75);
    return L == 0 ? n : n * 2.0 * sqrt(a);
}

/* np primitives with exponents a0[k] * zeta^2 and contraction coefficients d */
static void add_shell_n(omol *m, int *ns, int atom, int L, int np, const double *a0, double zeta,
                        const double *d, int bf0)
{
    oshell *s = &m->sh[*ns];
    int k, l;
    double self = 0.0;
    s->L = L; s->atom = atom; s->bf0 = bf0; s->np = np;
    for (k = 0; k < 3; k++) s->A[k] = m->R[3 * atom + k];
    for (k = 0; k < np; k++) {
        s->a[k] = a0[k] * zeta * zeta;
        s->c[k] = d[k] * prim_norm(L, s->a[k]);
    }
    /* renormalise so that <phi|phi> = 1 (x component for p) */
    for (k = 0; k < np; k++)
        for (l = 0; l < np; l++) {
            double p = s->a[k] + s->a[l];
            double v = pow(ORC_PI / p, 1.5);
            if (L == 1) v *= 0.5 / p;
            self += s->c[k] * s->c[l] * v;
        }
    for (k = 0; k < np; k++) s->c[k] /= sqrt(self);
    (*ns)++;
}

static void add_shell(omol *m, int *ns, int atom, int L, const double *a0, double zeta,
                      const double *d, int bf0)
{
    add_shell_n(m, ns, atom, L, 3, a0, zeta, d, bf0);
}

void orc_mol_free(void *h)
{
    omol *m = (omol *)h;
    if (!m) return;
    free(m->Z); free(m->R); free(m->sh); free(m->bf_shell); free(m->bf_comp);
    free(m);
}

/* index of a 6-31G heavy element in the tables (C, N, O), -1 otherwise */
static int g631_index(int Z) { return Z == 6 ? 0 : (Z == 7 ? 1 : (Z == 8 ? 2 : -1)); }

/* Returns NULL for unsupported elements, odd electron count, non-finite or
 * coincident (< 0.1 bohr) atoms.  basis: 0 = STO-3G (H, C, N, O, F),
 * 1 = 6-31G (H, C, N, O). */
void *orc_mol_new_basis(int natom, const int *Z, const double *xyz_ang, int charge, int basis)
{
    omol *m;
    int i, j, nsh = 0, nbf = 0, ns = 0, ne = 0;
    if (natom <= 0 || basis < 0 || basis > 1) return NULL;
    for (i = 0; i < natom; i++) {
        double z1 = 0.0, z2 = 0.0;
        if (!zeta_of(Z[i], &z1, &z2)) return NULL;
        if (basis == 1 && Z[i] != 1 && g631_index(Z[i]) < 0) return NULL;
        for (j = 0; j < 3; j++) if (!isfinite(xyz_ang[3 * i + j])) return NULL;
        if (basis == 0) {
            nsh += Z[i] == 1 ? 1 : 3;
            nbf += Z[i] == 1 ? 1 : 5;
        } else {
            nsh += Z[i] == 1 ? 2 : 5;
            nbf += Z[i] == 1 ? 2 : 9;
        }
        ne += Z[i];
    }
    ne -= charge;
    if (ne <= 0 || (ne & 1)) return NULL;
    m = (omol *)calloc(1, sizeof(omol));
    m->natom = natom; m->nshell = nsh; m->nbf = nbf; m->nelec = ne; m->nocc = ne / 2;
    m->Z = (int *)malloc(sizeof(int) * natom);
    m->R = (double *)malloc(sizeof(double) * 3 * natom);
    m->sh = (oshell *)calloc(nsh, sizeof(oshell));
    m->bf_shell = (int *)malloc(sizeof(int) * nbf);
    m->bf_comp = (int *)malloc(sizeof(int) * nbf);
    for (i = 0; i < natom; i++) {
        m->Z[i] = Z[i];
        for (j = 0; j < 3; j++) m->R[3 * i + j] = xyz_ang[3 * i + j] / ORC_BOHR_ANG;
    }
    for (i = 0; i < natom; i++)
        for (j = 0; j < i; j++) {
            double dx = m->R[3 * i] - m->R[3 * j], dy = m->R[3 * i + 1] - m->R[3 * j + 1],
                   dz = m->R[3 * i + 2] - m->R[3 * j + 2];
            if (sqrt(dx * dx + dy * dy + dz * dz) < 0.1) { orc_mol_free(m); return NULL; }
        }
    nbf = 0;
    for (i = 0; i < natom; i++) {
        double z1 = 0.0, z2 = 0.0;
        const double one = 1.0;
        const int ns0 = ns;
        zeta_of(Z[i], &z1, &z2);
        if (basis == 0) {
            add_shell(m, &ns, i, 0, STO1S_A, z1, STO1S_D, nbf); nbf += 1;
            if (Z[i] > 1) {
                add_shell(m, &ns, i, 0, STO2SP_A, z2, STO2S_D, nbf); nbf += 1;
                add_shell(m, &ns, i, 1, STO2SP_A, z2, STO2P_D, nbf); nbf += 3;
            }
            /* neutral-atom occupations: H 1s 1; 1s 2, 2s 2, 2p (Z-4)/3 each */
            m->sh[ns0].occ = Z[i] == 1 ? 1.0 : 2.0;
            if (Z[i] > 1) { m->sh[ns0 + 1].occ = 2.0; m->sh[ns0 + 2].occ = (Z[i] - 4) / 3.0; }
        } else if (Z[i] == 1) {
            add_shell_n(m, &ns, i, 0, 3, G631_H_A, 1.0, G631_H_D, nbf); nbf += 1;
            add_shell_n(m, &ns, i, 0, 1, &G631_H_A2, 1.0, &one, nbf); nbf += 1;
            /* the valence electron split evenly over the inner and outer s */
            m->sh[ns0].occ = 0.5; m->sh[ns0 + 1].occ = 0.5;
        } else {
            const int e = g631_index(Z[i]);
            add_shell_n(m, &ns, i, 0, 6, G631_1S[e].a, 1.0, G631_1S[e].d, nbf); nbf += 1;
            add_shell_n(m, &ns, i, 0, 3, G631_SP[e].a, 1.0, G631_SP[e].ds, nbf); nbf += 1;
            add_shell_n(m, &ns, i, 1, 3, G631_SP[e].a, 1.0, G631_SP[e].dp, nbf); nbf += 3;
            add_shell_n(m, &ns, i, 0, 1, &G631_SP[e].a3, 1.0, &one, nbf); nbf += 1;
            add_shell_n(m, &ns, i, 1, 1, &G631_SP[e].a3, 1.0, &one, nbf); nbf += 3;
            /* 1s 2; the valence split evenly over the inner and outer shells */
            m->sh[ns0].occ = 2.0;
            m->sh[ns0 + 1].occ = 1.0; m->sh[ns0 + 3].occ = 1.0;
            m->sh[ns0 + 2].occ = (Z[i] - 4) / 6.0; m->sh[ns0 + 4].occ = (Z[i] - 4) / 6.0;
        }
    }
    for (i = 0; i < nsh; i++) {
        oshell *s = &m->sh[i];
        if (s->L == 0) { m->bf_shell[s->bf0] = i; m->bf_comp[s->bf0] = 0; }
        else for (j = 0; j < 3; j++) { m->bf_shell[s->bf0 + j] = i; m->bf_comp[s->bf0 + j] = 1 + j; }
    }
    return m;
}

int orc_mol_info(void *h, int *nbf, int *nocc, int *nshell)
{
    omol *m = (omol *)h;
    *nbf = m->nbf; *nocc = m->nocc; *nshell = m->nshell;
    return 0;
}

void *orc_mol_new(int natom, const int *Z, const double *xyz_ang, int charge)
{
    return orc_mol_new_basis(natom, Z, xyz_ang, charge, 0);
}

/* Per-shell data for inspection: L, atom, bf0, primitive count, exponents[6],
 * coefs[6] (entries beyond the count are 0). */
void orc_shell(void *h, int s, int *L, int *atom, int *bf0, int *np, double *a, double *c)
{
    omol *m = (omol *)h;
    int k;
    *L = m->sh[s].L; *atom = m->sh[s].atom; *bf0 = m->sh[s].bf0; *np = m->sh[s].np;
    for (k = 0; k < 6; k++) {
        a[k] = k < m->sh[s].np ? m->sh[s].a[k] : 0.0;
        c[k] = k < m->sh[s].np ? m->sh[s].c[k] : 0.0;
    }
}

double orc_enuc(void *h)
{
    omol *m = (omol *)h;
    double e = 0.0;
    int i, j;
    for (i = 0; i < m->natom; i++)
        for (j = 0; j < i; j++) {
            double dx = m->R[3 * i] - m->R[3 * j], dy = m->R[3 * i + 1] - m->R[3 * j + 1],
                   dz = m->R[3 * i + 2] - m->R[3 * j + 2];
            e += m->Z[i] * m->Z[j] / sqrt(dx * dx + dy * dy + dz * dz);
        }
    return e;
}

/* Cartesian exponent triple of component c (0 = s, 1..3 = x,y,z) */
static void comp_lmn(int c, int *l)
{
    l[0] = l[1] = l[2] = 0;
    if (c > 0) l[c - 1] = 1;
}

/* ------------------------------------------------------------------ */
/* One-electron integrals, Obara-Saika                                 */
/* ------------------------------------------------------------------ */
/* 1D overlap S_ij for primitives with exponents a (on A) and b (on B), up to
 * i, j <= 2, by S_{i+1,j} = X_PA S_ij + (i S_{i-1,j} + j S_{i,j-1})/(2p),
 * S_{i,j+1} = X_PB S_ij + (...)/(2p); S_00 = sqrt(pi/p) exp(-mu X_AB^2). */
static void os_overlap1d(double a, double b, double A, double B, double S[4][4])
{
    double p = a + b, P = (a * A + b * B) / p, XPA = P - A, XPB = P - B;
    double mu = a * b / p;
    int i, j;
    for (i = 0; i < 4; i++) for (j = 0; j < 4; j++) S[i][j] = 0.0;
    S[0][0] = sqrt(ORC_PI / p) * exp(-mu * (A - B) * (A - B));
    for (i = 0; i < 3; i++) {
        S[i + 1][0] = XPA * S[i][0] + (i > 0 ? i * S[i - 1][0] : 0.0) / (2 * p);
    }
    for (j = 0; j < 3; j++)
        for (i = 0; i < 4; i++) {
            double v = XPB * S[i][j];
            if (i > 0) v += i * S[i - 1][j] / (2 * p);
            if (j > 0) v += j * S[i][j - 1] / (2 * p);
            S[i][j + 1] = v;
        }
}

/* 1D kinetic T_ij (i, j <= 1) from the overlap table (OS):
 * T_00 = [a - 2a^2 (X_PA^2 + 1/(2p))] S_00,
 * T_{i+1,j} = X_PA T_ij + (i T_{i-1,j} + j T_{i,j-1})/(2p) + (b/p)(2a S_{i+1,j} - i S_{i-1,j}),
 * T_{i,j+1} = X_PB T_ij + (i T_{i-1,j} + j T_{i,j-1})/(2p) + (a/p)(2b S_{i,j+1} - j S_{i,j-1}). */
static void os_kinetic1d(double a, double b, double A, double B, double S[4][4], double T[2][2])
{
    double p = a + b, P = (a * A + b * B) / p, XPA = P - A, XPB = P - B;
    T[0][0] = (a - 2 * a * a * (XPA * XPA + 1.0 / (2 * p))) * S[0][0];
    T[1][0] = XPA * T[0][0] + (b / p) * (2 * a * S[1][0]);
    T[0][1] = XPB * T[0][0] + (a / p) * (2 * b * S[0][1]);
    T[1][1] = XPB * T[1][0] + (1.0 * T[0][0]) / (2 * p) + (a / p) * (2 * b * S[1][1]);
}

/* Nuclear attraction: Theta^{(m)}(a, b) for one primitive pair and one
 * nucleus, OS recursion on the bra with horizontal transfer for b:
 * Theta^m_{a+1i,0} = PA_i Th^m_{a,0} - PC_i Th^{m+1}_{a,0}
 *                    + a_i/(2p) (Th^m_{a-1i,0} - Th^{m+1}_{a-1i,0}),
 * Theta^m_{00} = 2 pi/p K_AB F_m(p |PC|^2). */
typedef struct { double PA[3], PC[3], p; double base[4]; } nuc_ctx;

static double nuc_vrr(const nuc_ctx *c, const int *e, int m)
{
    int i, e1[3];
    double v;
    if (e[0] == 0 && e[1] == 0 && e[2] == 0) return c->base[m];
    i = e[0] ? 0 : (e[1] ? 1 : 2);
    e1[0] = e[0]; e1[1] = e[1]; e1[2] = e[2]; e1[i]--;
    v = c->PA[i] * nuc_vrr(c, e1, m) - c->PC[i] * nuc_vrr(c, e1, m + 1);
    if (e1[i] > 0) {
        int e2[3] = {e1[0], e1[1], e1[2]};
        e2[i]--;
        v += e1[i] / (2 * c->p) * (nuc_vrr(c, e2, m) - nuc_vrr(c, e2, m + 1));
    }
    return v;
}

static double nuc_hrr(const nuc_ctx *c, const int *a, const int *b, const double *AB)
{
    int i, a1[3], b1[3];
    if (b[0] == 0 && b[1] == 0 && b[2] == 0) return nuc_vrr(c, a, 0);
    i = b[0] ? 0 : (b[1] ? 1 : 2);
    a1[0] = a[0]; a1[1] = a[1]; a1[2] = a[2]; a1[i]++;
    b1[0] = b[0]; b1[1] = b[1]; b1[2] = b[2]; b1[i]--;
    return nuc_hrr(c, a1, b1, AB) + AB[i] * nuc_hrr(c, a, b1, AB);
}

/* S, T, V (all nuclei) in the AO basis, row-major N x N. */
void orc_int1e(void *h, double *S, double *T, double *V)
{
    omol *m = (omol *)h;
    int N = m->nbf, mu, nu;
    for (mu = 0; mu < N; mu++)
        for (nu = 0; nu <= mu; nu++) {
            const oshell *sa = &m->sh[m->bf_shell[mu]], *sb = &m->sh[m->bf_shell[nu]];
            int la[3], lb[3], k, l, d, C;
            double s = 0.0, t = 0.0, v = 0.0;
            comp_lmn(m->bf_comp[mu], la);
            comp_lmn(m->bf_comp[nu], lb);
            for (k = 0; k < sa->np; k++)
                for (l = 0; l < sb->np; l++) {
                    double a = sa->a[k], b = sb->a[l], p = a + b, cc = sa->c[k] * sb->c[l];
                    double S1[3][4][4], T1[3][2][2], P[3], AB[3], r2 = 0.0;
                    for (d = 0; d < 3; d++) {
                        os_overlap1d(a, b, sa->A[d], sb->A[d], S1[d]);
                        os_kinetic1d(a, b, sa->A[d], sb->A[d], S1[d], T1[d]);
                        P[d] = (a * sa->A[d] + b * sb->A[d]) / p;
                        AB[d] = sa->A[d] - sb->A[d];
                        r2 += AB[d] * AB[d];
                    }
                    s += cc * S1[0][la[0]][lb[0]] * S1[1][la[1]][lb[1]] * S1[2][la[2]][lb[2]];
                    t += cc * (T1[0][la[0]][lb[0]] * S1[1][la[1]][lb[1]] * S1[2][la[2]][lb[2]]
                             + S1[0][la[0]][lb[0]] * T1[1][la[1]][lb[1]] * S1[2][la[2]][lb[2]]
                             + S1[0][la[0]][lb[0]] * S1[1][la[1]][lb[1]] * T1[2][la[2]][lb[2]]);
                    for (C = 0; C < m->natom; C++) {
                        nuc_ctx c;
                        double pc2 = 0.0, F[4], K = exp(-a * b / p * r2);
                        int q;
                        c.p = p;
                        for (d = 0; d < 3; d++) {
                            c.PA[d] = P[d] - sa->A[d];
                            c.PC[d] = P[d] - m->R[3 * C + d];
                            pc2 += c.PC[d] * c.PC[d];
                        }
                        orc_boys(3, p * pc2, F);
                        for (q = 0; q < 4; q++) c.base[q] = 2.0 * ORC_PI / p * K * F[q];
                        v -= cc * m->Z[C] * nuc_hrr(&c, la, lb, AB);
                    }
                }
            S[mu * N + nu] = S[nu * N + mu] = s;
            T[mu * N + nu] = T[nu * N + mu] = t;
            V[mu * N + nu] = V[nu * N + mu] = v;
        }
}

/* ------------------------------------------------------------------ */
/* Electron repulsion integrals, Obara-Saika VRR + HRR                 */
/* ------------------------------------------------------------------ */
/* Cartesian triples with |e| <= 2 are indexed 0..9. */
static int cart_index(const int *e)
{
    int L = e[0] + e[1] + e[2];
    if (L == 0) return 0;
    if (L == 1) return 1 + (e[0] ? 0 : (e[1] ? 1 : 2));
    /* xx xy xz yy yz zz */
    if (e[0] == 2) return 4;
    if (e[0] == 1 && e[1] == 1) return 5;
    if (e[0] == 1 && e[2] == 1) return 6;
    if (e[1] == 2) return 7;
    if (e[1] == 1 && e[2] == 1) return 8;
    return 9;
}

typedef struct {
    double PA[3], WP[3], QC[3], WQ[3];
    double zeta, eta, rho;
    double base[5];
    double memo[10][10][5];
    unsigned char have[10][10][5];
} eri_ctx;

/* [e0|f0]^(m), Obara-Saika vertical recurrence (electron 1 first, then 2):
 * [e+1i,0|f0]^m = PA_i [e0|f0]^m + WP_i [e0|f0]^{m+1}
 *   + e_i/(2 zeta) ([e-1i,0|f0]^m - rho/zeta [e-1i,0|f0]^{m+1})
 *   + f_i/(2(zeta+eta)) [e0|f-1i,0]^{m+1},
 * [00|f+1i,0]^m = QC_i [00|f0]^m + WQ_i [00|f0]^{m+1}
 *   + f_i/(2 eta) ([00|f-1i,0]^m - rho/eta [00|f-1i,0]^{m+1}). */
static double eri_vrr(eri_ctx *c, const int *e, const int *f, int m)
{
    int ie = cart_index(e), jf = cart_index(f), i;
    double v;
    if (c->have[ie][jf][m]) return c->memo[ie][jf][m];
    if (e[0] + e[1] + e[2] > 0) {
        int e1[3] = {e[0], e[1], e[2]};
        i = e[0] ? 0 : (e[1] ? 1 : 2);
        e1[i]--;
        v = c->PA[i] * eri_vrr(c, e1, f, m) + c->WP[i] * eri_vrr(c, e1, f, m + 1);
        if (e1[i] > 0) {
            int e2[3] = {e1[0], e1[1], e1[2]};
            e2[i]--;
            v += e1[i] / (2 * c->zeta) * (eri_vrr(c, e2, f, m) - c->rho / c->zeta * eri_vrr(c, e2, f, m + 1));
        }
        if (f[i] > 0) {
            int f1[3] = {f[0], f[1], f[2]};
            f1[i]--;
            v += f[i] / (2 * (c->zeta + c->eta)) * eri_vrr(c, e1, f1, m + 1);
        }
    } else if (f[0] + f[1] + f[2] > 0) {
        int f1[3] = {f[0], f[1], f[2]};
        i = f[0] ? 0 : (f[1] ? 1 : 2);
        f1[i]--;
        v = c->QC[i] * eri_vrr(c, e, f1, m) + c->WQ[i] * eri_vrr(c, e, f1, m + 1);
        if (f1[i] > 0) {
            int f2[3] = {f1[0], f1[1], f1[2]};
            f2[i]--;
            v += f1[i] / (2 * c->eta) * (eri_vrr(c, e, f2, m) - c->rho / c->eta * eri_vrr(c, e, f2, m + 1));
        }
    } else {
        v = c->base[m];
    }
    c->have[ie][jf][m] = 1;
    c->memo[ie][jf][m] = v;
    return v;
}

/* contracted [e0|f0] table for one shell quartet, then HRR:
 * (a,b+1i|cd) = (a+1i,b|cd) + AB_i (ab|cd);  (ab|c,d+1i) = (ab|c+1i,d) + CD_i (ab|cd). */
typedef struct { double t[10][10]; double AB[3], CD[3]; } eri_contracted;

static double eri_hrr(const eri_contracted *q, const int *a, const int *b, const int *c, const int *d)
{
    int i;
    if (b[0] + b[1] + b[2] > 0) {
        int a1[3] = {a[0], a[1], a[2]}, b1[3] = {b[0], b[1], b[2]};
        i = b[0] ? 0 : (b[1] ? 1 : 2);
        a1[i]++; b1[i]--;
        return eri_hrr(q, a1, b1, c, d) + q->AB[i] * eri_hrr(q, a, b1, c, d);
    }
    if (d[0] + d[1] + d[2] > 0) {
        int c1[3] = {c[0], c[1], c[2]}, d1[3] = {d[0], d[1], d[2]};
        i = d[0] ? 0 : (d[1] ? 1 : 2);
        c1[i]++; d1[i]--;
        return eri_hrr(q, a, b, c1, d1) + q->CD[i] * eri_hrr(q, a, b, c, d1);
    }
    return q->t[cart_index(a)][cart_index(c)];
}

static const int CART[10][3] = {{0,0,0},{1,0,0},{0,1,0},{0,0,1},{2,0,0},{1,1,0},{1,0,1},{0,2,0},{0,1,1},{0,0,2}};

/* Block of contracted (ab|cd) over the components of shells a, b, c, d:
 * out[((i*nb + j)*nc + k)*nd + l]. */
static void eri_shell_quartet(const omol *m, int ia, int ib, int ic, int id, double *out)
{
    const oshell *A = &m->sh[ia], *B = &m->sh[ib], *C = &m->sh[ic], *D = &m->sh[id];
    eri_contracted q;
    int La = A->L, Lb = B->L, Lc = C->L, Ld = D->L;
    int pa, pb, pc, pd, d, e, f;
    int na = La ? 3 : 1, nb = Lb ? 3 : 1, nc = Lc ? 3 : 1, nd = Ld ? 3 : 1;
    double rab2 = 0.0, rcd2 = 0.0;
    memset(&q, 0, sizeof(q));
    for (d = 0; d < 3; d++) {
        q.AB[d] = A->A[d] - B->A[d];
        q.CD[d] = C->A[d] - D->A[d];
        rab2 += q.AB[d] * q.AB[d];
        rcd2 += q.CD[d] * q.CD[d];
    }
    for (pa = 0; pa < A->np; pa++)
        for (pb = 0; pb < B->np; pb++)
            for (pc = 0; pc < C->np; pc++)
                for (pd = 0; pd < D->np; pd++) {
                    double a = A->a[pa], b = B->a[pb], c = C->a[pc], dd = D->a[pd];
                    double zeta = a + b, eta = c + dd, rho = zeta * eta / (zeta + eta);
                    double P[3], Q[3], W[3], pq2 = 0.0, F[5], pref;
                    double cc = A->c[pa] * B->c[pb] * C->c[pc] * D->c[pd];
                    eri_ctx x;
                    int Lt = La + Lb + Lc + Ld, k;
                    memset(x.have, 0, sizeof(x.have));
                    for (d = 0; d < 3; d++) {
                        P[d] = (a * A->A[d] + b * B->A[d]) / zeta;
                        Q[d] = (c * C->A[d] + dd * D->A[d]) / eta;
                        W[d] = (zeta * P[d] + eta * Q[d]) / (zeta + eta);
                        x.PA[d] = P[d] - A->A[d];
                        x.WP[d] = W[d] - P[d];
                        x.QC[d] = Q[d] - C->A[d];
                        x.WQ[d] = W[d] - Q[d];
                        pq2 += (P[d] - Q[d]) * (P[d] - Q[d]);
                    }
                    x.zeta = zeta; x.eta = eta; x.rho = rho;
                    orc_boys(Lt, rho * pq2, F);
                    pref = 2.0 * pow(ORC_PI, 2.5) / (zeta * eta * sqrt(zeta + eta))
                         * exp(-a * b / zeta * rab2) * exp(-c * dd / eta * rcd2);
                    for (k = 0; k <= Lt; k++) x.base[k] = pref * F[k];
                    for (e = 0; e < 10; e++) {
                        int le = CART[e][0] + CART[e][1] + CART[e][2];
                        if (le < La || le > La + Lb) continue;
                        for (f = 0; f < 10; f++) {
                            int lf = CART[f][0] + CART[f][1] + CART[f][2];
                            if (lf < Lc || lf > Lc + Ld) continue;
                            q.t[e][f] += cc * eri_vrr(&x, CART[e], CART[f], 0);
                        }
                    }
                }
    {
        int i, j, k, l;
        for (i = 0; i < na; i++)
            for (j = 0; j < nb; j++)
                for (k = 0; k < nc; k++)
                    for (l = 0; l < nd; l++) {
                        int ca[3], cb[3], cc3[3], cd[3];
                        comp_lmn(La ? 1 + i : 0, ca);
                        comp_lmn(Lb ? 1 + j : 0, cb);
                        comp_lmn(Lc ? 1 + k : 0, cc3);
                        comp_lmn(Ld ? 1 + l : 0, cd);
                        out[((i * nb + j) * nc + k) * nd + l] = eri_hrr(&q, ca, cb, cc3, cd);
                    }
    }
}

static long pair_index(int i, int j) { return i >= j ? (long)i * (i + 1) / 2 + j : (long)j * (j + 1) / 2 + i; }

static long quartet_index(int i, int j, int k, int l)
{
    long ij = pair_index(i, j), kl = pair_index(k, l);
    return ij >= kl ? ij * (ij + 1) / 2 + kl : kl * (kl + 1) / 2 + ij;
}

long orc_n_eri(void *h)
{
    omol *m = (omol *)h;
    long np = (long)m->nbf * (m->nbf + 1) / 2;
    return np * (np + 1) / 2;
}

/* All unique (ij|kl), i>=j, k>=l, ij>=kl, at index ij(ij+1)/2 + kl with
 * ij = i(i+1)/2 + j.  No screening. */
void orc_eri(void *h, double *out)
{
    omol *m = (omol *)h;
    int a, b, c, d;
    double blk[81];
    for (a = 0; a < m->nshell; a++)
        for (b = 0; b <= a; b++)
            for (c = 0; c <= a; c++)
                for (d = 0; d <= c; d++) {
                    const oshell *A = &m->sh[a], *B = &m->sh[b], *C = &m->sh[c], *D = &m->sh[d];
                    int na = A->L ? 3 : 1, nb = B->L ? 3 : 1, nc = C->L ? 3 : 1, nd = D->L ? 3 : 1;
                    int i, j, k, l;
                    if (c == a && d > b) continue;
                    eri_shell_quartet(m, a, b, c, d, blk);
                    for (i = 0; i < na; i++)
                        for (j = 0; j < nb; j++)
                            for (k = 0; k < nc; k++)
                                for (l = 0; l < nd; l++)
                                    out[quartet_index(A->bf0 + i, B->bf0 + j, C->bf0 + k, D->bf0 + l)] =
                                        blk[((i * nb + j) * nc + k) * nd + l];
                }
}

/* One integral (ij|kl) for sampled checks at full size. */
double orc_eri_one(void *h, int i, int j, int k, int l)
{
    omol *m = (omol *)h;
    int a = m->bf_shell[i], b = m->bf_shell[j], c = m->bf_shell[k], d = m->bf_shell[l];
    int nb = m->sh[b].L ? 3 : 1, nc = m->sh[c].L ? 3 : 1, nd = m->sh[d].L ? 3 : 1;
    int ci = i - m->sh[a].bf0, cj = j - m->sh[b].bf0, ck = k - m->sh[c].bf0, cl = l - m->sh[d].bf0;
    double blk[81];
    eri_shell_quartet(m, a, b, c, d, blk);
    return blk[((ci * nb + cj) * nc + ck) * nd + cl];
}

/* J_ij = sum_kl (ij|kl) P_kl and K_ij = sum_kl (ik|jl) P_kl from the packed
 * unique list: every unique integral is expanded to the distinct index
 * quadruples of its 8-element permutation orbit (paper section 3.2, the
 * footnote on the 8-fold symmetry) and each quadruple (a,b,c,d) adds
 * I P_cd to J_ab and I P_bd to K_ac -- the definition summed over N^4. */
void orc_jk(void *h, const double *eri, const double *P, double *J, double *K)
{
    omol *m = (omol *)h;
    int N = m->nbf, i, j, k, l;
    long idx = 0;
    memset(J, 0, sizeof(double) * N * N);
    memset(K, 0, sizeof(double) * N * N);
    for (i = 0; i < N; i++)
        for (j = 0; j <= i; j++)
            for (k = 0; k <= i; k++)
                for (l = 0; l <= (k == i ? j : k); l++) {
                    double I = eri[quartet_index(i, j, k, l)];
                    int perm[8][4] = {{i,j,k,l},{j,i,k,l},{i,j,l,k},{j,i,l,k},
                                      {k,l,i,j},{l,k,i,j},{k,l,j,i},{l,k,j,i}};
                    int p, q, dup;
                    (void)idx;
                    for (p = 0; p < 8; p++) {
                        dup = 0;
                        for (q = 0; q < p; q++)
                            if (perm[q][0] == perm[p][0] && perm[q][1] == perm[p][1] &&
                                perm[q][2] == perm[p][2] && perm[q][3] == perm[p][3]) { dup = 1; break; }
                        if (dup) continue;
                        {
                            int a = perm[p][0], b = perm[p][1], c = perm[p][2], d = perm[p][3];
                            J[a * N + b] += I * P[c * N + d];
                            K[a * N + c] += I * P[b * N + d];
                        }
                    }
                }
}

/* ------------------------------------------------------------------ */
/* Integration grid                                                    */
/* ------------------------------------------------------------------ */
/* Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_n. */
void orc_gauss_legendre(int n, double *x, double *w)
{
    int i, it, k;
    for (i = 0; i < n; i++) {
        double z = cos(ORC_PI * (i + 0.75) / (n + 0.5)), pp = 0.0;
        for (it = 0; it < 100; it++) {
            double p0 = 1.0, p1 = z, dz;
            for (k = 2; k <= n; k++) {
                double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1; p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            pp = n * (z * p1 - p0) / (z * z - 1.0);
            dz = p1 / pp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        {
            double p0 = 1.0, p1 = z;
            for (k = 2; k <= n; k++) {
                double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1; p1 = p2;
            }
            pp = n * (z * p1 - p0) / (z * z - 1.0);
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * pp * pp);
    }
}

/* Treutler-Ahlrichs M4 radial rule, xi = 1, alpha = 0.6:
 * r(x) = (xi/ln 2)(1+x)^0.6 ln(2/(1-x)), x_i = cos(i pi/(n+1)),
 * w_i = pi/(n+1) sin(i pi/(n+1)) r'(x_i) r_i^2  (includes the r^2 Jacobian). */
void orc_radial(int n, double *r, double *w)
{
    int i;
    double xi = 1.0, al = 0.6, ln2 = log(2.0);
    for (i = 1; i <= n; i++) {
        double th = i * ORC_PI / (n + 1), x = cos(th);
        double rr = xi / ln2 * pow(1 + x, al) * log(2.0 / (1 - x));
        double dr = xi / ln2 * (al * pow(1 + x, al - 1) * log(2.0 / (1 - x)) + pow(1 + x, al) / (1 - x));
        r[i - 1] = rr;
        w[i - 1] = ORC_PI / (n + 1) * sin(th) * dr * rr * rr;
    }
}

static double becke_step(double mu)
{
    int k;
    for (k = 0; k < 3; k++) mu = 1.5 * mu - 0.5 * mu * mu * mu;
    return 0.5 * (1.0 - mu);
}

/* Becke fuzzy-cell weight of atom A at point p: P_A / sum_C P_C with
 * P_A = prod_{B != A} s(mu_AB), mu_AB = (|p-R_A| - |p-R_B|)/|R_A-R_B|. */
static double becke_weight(const omol *m, int A, const double *p)
{
    int a, b;
    double num = 0.0, den = 0.0;
    for (a = 0; a < m->natom; a++) {
        double Pa = 1.0, ra, dx, dy, dz;
        dx = p[0] - m->R[3 * a]; dy = p[1] - m->R[3 * a + 1]; dz = p[2] - m->R[3 * a + 2];
        ra = sqrt(dx * dx + dy * dy + dz * dz);
        for (b = 0; b < m->natom; b++) {
            double rb, rab;
            if (b == a) continue;
            dx = p[0] - m->R[3 * b]; dy = p[1] - m->R[3 * b + 1]; dz = p[2] - m->R[3 * b + 2];
            rb = sqrt(dx * dx + dy * dy + dz * dz);
            dx = m->R[3 * a] - m->R[3 * b]; dy = m->R[3 * a + 1] - m->R[3 * b + 1]; dz = m->R[3 * a + 2] - m->R[3 * b + 2];
            rab = sqrt(dx * dx + dy * dy + dz * dz);
            Pa *= becke_step((ra - rb) / rab);
        }
        if (a == A) num = Pa;
        den += Pa;
    }
    return num / den;
}

long orc_grid_size(void *h, int nrad, int nth, int nph)
{
    omol *m = (omol *)h;
    return (long)m->natom * nrad * nth * nph;
}

/* Grid points [G][4] = (x, y, z, w) in bohr; atom-major, then radial
 * (outermost first), then theta (Gauss-Legendre order), then phi_k = 2 pi k/nph. */
void orc_grid(void *h, int nrad, int nth, int nph, double *out)
{
    omol *m = (omol *)h;
    double *r = malloc(sizeof(double) * nrad), *wr = malloc(sizeof(double) * nrad);
    double *ct = malloc(sizeof(double) * nth), *wt = malloc(sizeof(double) * nth);
    long g = 0;
    int A, i, j, k;
    orc_radial(nrad, r, wr);
    orc_gauss_legendre(nth, ct, wt);
    for (A = 0; A < m->natom; A++)
        for (i = 0; i < nrad; i++)
            for (j = 0; j < nth; j++)
                for (k = 0; k < nph; k++) {
                    double st = sqrt(1.0 - ct[j] * ct[j]), ph = 2.0 * ORC_PI * k / nph, p[3];
                    p[0] = m->R[3 * A] + r[i] * st * cos(ph);
                    p[1] = m->R[3 * A + 1] + r[i] * st * sin(ph);
                    p[2] = m->R[3 * A + 2] + r[i] * ct[j];
                    out[4 * g] = p[0]; out[4 * g + 1] = p[1]; out[4 * g + 2] = p[2];
                    out[4 * g + 3] = wr[i] * wt[j] * (2.0 * ORC_PI / nph) * becke_weight(m, A, p);
                    g++;
                }
    free(r); free(wr); free(ct); free(wt);
}

/* ------------------------------------------------------------------ */
/* AO values and gradients                                             */
/* ------------------------------------------------------------------ */
/* phi[4][N]: value, d/dx, d/dy, d/dz of every AO at point p. */
static void ao_point(const omol *m, const double *p, double *phi)
{
    int N = m->nbf, s, k;
    for (s = 0; s < m->nshell; s++) {
        const oshell *S = &m->sh[s];
        double d[3] = {p[0] - S->A[0], p[1] - S->A[1], p[2] - S->A[2]};
        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2], R = 0.0, dR = 0.0;
        for (k = 0; k < S->np; k++) {
            double e = S->c[k] * exp(-S->a[k] * r2);
            R += e;
            dR += -2.0 * S->a[k] * e;   /* (1/r) dR/dr */
        }
        if (S->L == 0) {
            int mu = S->bf0;
            phi[mu] = R;
            for (k = 0; k < 3; k++) phi[(k + 1) * N + mu] = dR * d[k];
        } else {
            int c;
            for (c = 0; c < 3; c++) {
                int mu = S->bf0 + c;
                phi[mu] = d[c] * R;
                for (k = 0; k < 3; k++)
                    phi[(k + 1) * N + mu] = (k == c ? R : 0.0) + d[c] * d[k] * dR;
            }
        }
    }
}

void orc_ao(void *h, long npt, const double *xyz, double *phi)
{
    omol *m = (omol *)h;
    long g;
    for (g = 0; g < npt; g++) ao_point(m, xyz + 3 * g, phi + (long)4 * m->nbf * g);
}

/* ------------------------------------------------------------------ */
/* B3LYP, closed shell, energy density per volume and its derivatives  */
/* with respect to rho and sigma = |grad rho|^2                        */
/* ------------------------------------------------------------------ */
#define XC_HF 0
#define XC_B3LYP 1      /* VWN RPA fit */
#define XC_B3LYP5 2     /* VWN5 */
#define RHO_CUT 1e-12

/* Slater exchange: e = -(3/4)(3/pi)^(1/3) rho^(4/3) */
static void slater(double rho, double *e, double *vr)
{
    double c = 0.75 * cbrt(3.0 / ORC_PI), r13 = cbrt(rho);
    *e = -c * rho * r13;
    *vr = -4.0 / 3.0 * c * r13;
}

/* Becke 88 exchange (includes the LDA part), closed shell:
 * e = 2 e_s(rho/2, sqrt(sigma)/2), e_s(r, g) = -r^(4/3) [Cx + beta x^2 / D],
 * x = g / r^(4/3), D = 1 + 6 beta x asinh x, Cx = (3/2)(3/(4 pi))^(1/3). */
static void becke88(double rho, double sigma, double *e, double *vr, double *vs)
{
    const double beta = 0.0042, Cx = 1.5 * cbrt(3.0 / (4.0 * ORC_PI));
    double rs = 0.5 * rho, r13 = cbrt(rs), r43 = rs * r13;
    double gs = 0.5 * sqrt(sigma), x = gs / r43;
    double ash = asinh(x), D = 1.0 + 6.0 * beta * x * ash;
    double Dp = 6.0 * beta * (ash + x / sqrt(1.0 + x * x));
    double g = x * x / D;
    double gp_over_x = (2.0 * D - x * Dp) / (D * D);   /* g'(x)/x */
    double es = -r43 * (Cx + beta * g);
    double des_drs = -4.0 / 3.0 * r13 * (Cx + beta * (g - x * x * gp_over_x));
    *e = 2.0 * es;
    *vr = des_drs;                                   /* 2 * des/drs * 1/2 */
    *vs = -beta * gp_over_x / (4.0 * r43);           /* d e / d sigma */
}

/* VWN correlation (paramagnetic), e = rho eps(x), x = sqrt(rs):
 * eps = A { ln(x^2/X) + 2b/Q atan(Q/(2x+b))
 *           - b x0/X(x0) [ ln((x-x0)^2/X) + 2(b+2x0)/Q atan(Q/(2x+b)) ] },
 * X = x^2 + b x + c, Q = sqrt(4c - b^2);  v = eps - (x/6) deps/dx. */
static void vwn(double rho, int variant, double *e, double *vr)
{
    const double A = 0.0310907;
    double b, c, x0;
    double rs, x, X, X0, Q, at, eps, deps;
    if (variant == XC_B3LYP5) { b = 3.72744; c = 12.9352; x0 = -0.10498; }
    else { b = 13.0720; c = 42.7198; x0 = -0.409286; }
    rs = cbrt(3.0 / (4.0 * ORC_PI * rho));
    x = sqrt(rs);
    X = x * x + b * x + c;
    X0 = x0 * x0 + b * x0 + c;
    Q = sqrt(4.0 * c - b * b);
    at = atan(Q / (2.0 * x + b));
    eps = A * (log(x * x / X) + 2.0 * b / Q * at
               - b * x0 / X0 * (log((x - x0) * (x - x0) / X) + 2.0 * (b + 2.0 * x0) / Q * at));
    deps = A * (2.0 / x - (2.0 * x + b) / X - b / X
                - b * x0 / X0 * (2.0 / (x - x0) - (2.0 * x + b) / X - (b + 2.0 * x0) / X));
    *e = rho * eps;
    *vr = eps - x / 6.0 * deps;
}

/* LYP correlation, closed shell, gradient-only form (Miehlich et al. 1989)
 * specialised to rho_a = rho_b = rho/2:
 * e = -a rho/den - a b C_F E/den rho + (a b/72) E/den rho^(-5/3) sigma (3 + 7 delta),
 * t = rho^(-1/3), den = 1 + d t, E = exp(-c t), delta = c t + d t/den,
 * C_F = (3/10)(3 pi^2)^(2/3). */
static void lyp(double rho, double sigma, double *e, double *vr, double *vs)
{
    const double a = 0.04918, b = 0.132, c = 0.2533, d = 0.349;
    const double CF = 0.3 * pow(3.0 * ORC_PI * ORC_PI, 2.0 / 3.0);
    double t = 1.0 / cbrt(rho), den = 1.0 + d * t, E = exp(-c * t);
    double delta = c * t + d * t / den;
    double r53 = pow(rho, -5.0 / 3.0), r83 = r53 / rho;
    double Eden = E / den;
    double t1 = -a * rho / den;
    double t2 = -a * b * CF * Eden * rho;
    double t3 = a * b / 72.0 * Eden * r53 * sigma * (3.0 + 7.0 * delta);
    double dt1 = -a / den - a * d * t / (3.0 * den * den);
    double dt2 = -a * b * CF * Eden * (1.0 + delta / 3.0);
    double dt3 = a * b / 72.0 * sigma * Eden * r83 / 3.0
               * (7.0 * delta * delta - 39.0 * delta - 15.0 + 7.0 * d * d * t * t / (den * den));
    *e = t1 + t2 + t3;
    *vr = dt1 + dt2 + dt3;
    *vs = a * b / 72.0 * Eden * r53 * (3.0 + 7.0 * delta);
}

/* Per point: e (energy per volume), v_rho, v_sigma.  xc = 1 (B3LYP, VWN RPA)
 * or 2 (VWN5); 0 gives zeros (Hartree-Fock).  Individual pieces can be asked
 * for with xc = 10 (Slater), 11 (B88), 12 (VWN RPA), 13 (VWN5), 14 (LYP). */
void orc_functional(int xc, long n, const double *rho, const double *sigma,
                    double *e, double *vr, double *vs)
{
    long g;
    for (g = 0; g < n; g++) {
        double r = rho[g], s = sigma[g] < 0 ? 0.0 : sigma[g];
        double es, vs_, eb, vb, sb, ev, vv, el, vl, sl;
        e[g] = vr[g] = vs[g] = 0.0;
        if (xc == XC_HF || r < RHO_CUT) continue;
        switch (xc) {
        case 10: slater(r, &e[g], &vr[g]); continue;
        case 11: becke88(r, s, &e[g], &vr[g], &vs[g]); continue;
        case 12: vwn(r, XC_B3LYP, &e[g], &vr[g]); continue;
        case 13: vwn(r, XC_B3LYP5, &e[g], &vr[g]); continue;
        case 14: lyp(r, s, &e[g], &vr[g], &vs[g]); continue;
        default: break;
        }
        slater(r, &es, &vs_);
        becke88(r, s, &eb, &vb, &sb);
        vwn(r, xc, &ev, &vv);
        lyp(r, s, &el, &vl, &sl);
        e[g] = 0.08 * es + 0.72 * eb + 0.19 * ev + 0.81 * el;
        vr[g] = 0.08 * vs_ + 0.72 * vb + 0.19 * vv + 0.81 * vl;
        vs[g] = 0.72 * sb + 0.81 * sl;
    }
}

/* Neumaier compensated accumulator */
typedef struct { double s, c; } ksum;
static void ksum_add(ksum *k, double x)
{
    double t = k->s + x;
    if (fabs(k->s) >= fabs(x)) k->c += (k->s - t) + x;
    else k->c += (x - t) + k->s;
    k->s = t;
}
static double ksum_get(const ksum *k) { return k->s + k->c; }

/* E_xc = sum_g w_g e_g and
 * V_mn = sum_g w_g [v_rho phi_m phi_n + 2 v_sigma grad rho . grad(phi_m phi_n)]
 * with rho = sum_mn P_mn phi_m phi_n.  xyzw is [G][4]. */
double orc_xc(void *h, int xc, long npt, const double *xyzw, const double *P, double *V)
{
    omol *m = (omol *)h;
    int N = m->nbf, mu, nu;
    double *phi = malloc(sizeof(double) * 4 * N), *X = malloc(sizeof(double) * N),
           *W = malloc(sizeof(double) * N);
    ksum ex = {0.0, 0.0};
    long g;
    memset(V, 0, sizeof(double) * N * N);
    if (xc == XC_HF) { free(phi); free(X); free(W); return 0.0; }
    for (g = 0; g < npt; g++) {
        const double *p = xyzw + 4 * g;
        double w = p[3], rho = 0.0, gr[3] = {0.0, 0.0, 0.0}, sigma, e, vr, vs;
        ao_point(m, p, phi);
        for (mu = 0; mu < N; mu++) {
            double s = 0.0;
            for (nu = 0; nu < N; nu++) s += P[mu * N + nu] * phi[nu];
            X[mu] = s;
        }
        for (mu = 0; mu < N; mu++) {
            rho += phi[mu] * X[mu];
            gr[0] += 2.0 * X[mu] * phi[N + mu];
            gr[1] += 2.0 * X[mu] * phi[2 * N + mu];
            gr[2] += 2.0 * X[mu] * phi[3 * N + mu];
        }
        if (rho < RHO_CUT) continue;
        sigma = gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2];
        orc_functional(xc, 1, &rho, &sigma, &e, &vr, &vs);
        ksum_add(&ex, w * e);
        for (mu = 0; mu < N; mu++)
            W[mu] = w * (0.5 * vr * phi[mu]
                         + 2.0 * vs * (gr[0] * phi[N + mu] + gr[1] * phi[2 * N + mu] + gr[2] * phi[3 * N + mu]));
        for (mu = 0; mu < N; mu++)
            for (nu = 0; nu <= mu; nu++)
                V[mu * N + nu] += phi[mu] * W[nu] + W[mu] * phi[nu];
    }
    for (mu = 0; mu < N; mu++)
        for (nu = 0; nu < mu; nu++) V[nu * N + mu] = V[mu * N + nu];
    free(phi); free(X); free(W);
    return ksum_get(&ex);
}

/* ------------------------------------------------------------------ */
/* dense linear algebra                                                */
/* ------------------------------------------------------------------ */
/* Symmetric eigenproblem by cyclic Jacobi rotations.  w ascending, columns
 * of V (row-major, V[i*n + k] = component i of vector k) the eigenvectors. */
int orc_eigh(int n, const double *Ain, double *w, double *V)
{
    double *A = malloc(sizeof(double) * n * n);
    int i, j, k, p, q, sweep;
    memcpy(A, Ain, sizeof(double) * n * n);
    for (i = 0; i < n; i++) for (j = 0; j < n; j++) V[i * n + j] = (i == j);
    for (sweep = 0; sweep < 100; sweep++) {
        double off = 0.0, tot = 0.0;
        for (i = 0; i < n; i++)
            for (j = 0; j < n; j++) {
                tot += A[i * n + j] * A[i * n + j];
                if (i != j) off += A[i * n + j] * A[i * n + j];
            }
        if (off <= 1e-30 * tot || off == 0.0) break;
        for (p = 0; p < n - 1; p++)
            for (q = p + 1; q < n; q++) {
                double apq = A[p * n + q], app, aqq, th, t, c, s;
                if (apq == 0.0) continue;
                app = A[p * n + p]; aqq = A[q * n + q];
                th = (aqq - app) / (2.0 * apq);
                t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                c = 1.0 / sqrt(t * t + 1.0); s = t * c;
                for (k = 0; k < n; k++) {           /* columns p, q */
                    double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - s * akq;
                    A[k * n + q] = s * akp + c * akq;
                }
                for (k = 0; k < n; k++) {           /* rows p, q */
                    double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - s * aqk;
                    A[q * n + k] = s * apk + c * aqk;
                }
                for (k = 0; k < n; k++) {
                    double vkp = V[k * n + p], vkq = V[k * n + q];
                    V[k * n + p] = c * vkp - s * vkq;
                    V[k * n + q] = s * vkp + c * vkq;
                }
            }
    }
    for (i = 0; i < n; i++) w[i] = A[i * n + i];
    /* selection sort, ascending */
    for (i = 0; i < n; i++) {
        int mi = i;
        for (j = i + 1; j < n; j++) if (w[j] < w[mi]) mi = j;
        if (mi != i) {
            double t = w[i]; w[i] = w[mi]; w[mi] = t;
            for (k = 0; k < n; k++) { t = V[k * n + i]; V[k * n + i] = V[k * n + mi]; V[k * n + mi] = t; }
        }
    }
    free(A);
    return 0;
}

static void matmul(int n, const double *A, int ta, const double *B, int tb, double *C)
{
    int i, j, k;
    for (i = 0; i < n; i++)
        for (j = 0; j < n; j++) {
            double s = 0.0;
            for (k = 0; k < n; k++)
                s += (ta ? A[k * n + i] : A[i * n + k]) * (tb ? B[j * n + k] : B[k * n + j]);
            C[i * n + j] = s;
        }
}

/* Solve the (n+1) bordered DIIS system [B -1; -1^T 0][c; l] = [0; -1] by
 * Gaussian elimination with partial pivoting.  Returns 0 if a pivot falls
 * below 1e-12 max|B| (singular: the caller drops the oldest vector). */
static int diis_solve(int n, const double *B, double *c)
{
    int M = n + 1, i, j, k;
    double *a = malloc(sizeof(double) * M * (M + 1)), bmax = 0.0;
    for (i = 0; i < n; i++) for (j = 0; j < n; j++) if (fabs(B[i * n + j]) > bmax) bmax = fabs(B[i * n + j]);
    for (i = 0; i < M; i++) {
        for (j = 0; j < M; j++) {
            double v;
            if (i < n && j < n) v = B[i * n + j];
            else if (i == n && j == n) v = 0.0;
            else v = -1.0;
            a[i * (M + 1) + j] = v;
        }
        a[i * (M + 1) + M] = (i == n) ? -1.0 : 0.0;
    }
    for (k = 0; k < M; k++) {
        int piv = k;
        double t;
        for (i = k + 1; i < M; i++) if (fabs(a[i * (M + 1) + k]) > fabs(a[piv * (M + 1) + k])) piv = i;
        if (fabs(a[piv * (M + 1) + k]) < 1e-12 * bmax) { free(a); return 0; }
        if (piv != k)
            for (j = 0; j <= M; j++) { t = a[k * (M + 1) + j]; a[k * (M + 1) + j] = a[piv * (M + 1) + j]; a[piv * (M + 1) + j] = t; }
        for (i = k + 1; i < M; i++) {
            double f = a[i * (M + 1) + k] / a[k * (M + 1) + k];
            for (j = k; j <= M; j++) a[i * (M + 1) + j] -= f * a[k * (M + 1) + j];
        }
    }
    for (i = M - 1; i >= 0; i--) {
        double s = a[i * (M + 1) + M];
        for (j = i + 1; j < M; j++) s -= a[i * (M + 1) + j] * c[j];
        c[i] = s / a[i * (M + 1) + i];
    }
    free(a);
    return 1;
}

/* ------------------------------------------------------------------ */
/* SCF                                                                 */
/* ------------------------------------------------------------------ */
/* status codes */
#define ST_CONVERGED 1
#define ST_MAXITER 2
#define ST_DIVERGED 3
#define ST_INVALID 4

/* Restricted Kohn-Sham SCF (paper section 3.1: iteration 0 precomputes
 * V, T, S, ERIs and the initial orbitals; iteration i forms rho_i, V_XC,
 * J, K and solves the generalised eigenproblem).
 *   X = S^-1/2 (Loewdin); initial density: atomic occupations (guess 0) or
 *   diagonalise X^T H X (guess 1); P = 2 C_occ C_occ^T.
 *   iteration k: F_k = H + J[P] - (a0/2) K[P] + V_xc[P],
 *     E_k = tr(PH) + 1/2 tr(PJ) - a0/4 tr(PK) + E_xc + E_nn,
 *     e_k = X^T (F P S - S P F) X;  converged when k > 1,
 *     |E_k - E_{k-1}| < e_tol and max|e_k| < comm_tol;
 *     else DIIS over the last `diis_space` (F, e) pairs, diagonalise
 *     X^T Fbar X, new P from the lowest nocc orbitals.
 *   On exit eps are the eigenvalues of X^T F_k X (no extrapolation) and P
 *   is the density that produced F_k.
 * Eterms[6] = {tr PH, 1/2 tr PJ, -a0/4 tr PK, E_xc, E_nn, E}. */
int orc_scf(void *h, int xc, int nrad, int nth, int nph, double e_tol, double comm_tol,
            int max_iter, int diis_space, int guess, double *E_out, double *eps, double *P_out,
            int *niter, int *status, double *Eterms)
{
    omol *m = (omol *)h;
    int N = m->nbf, nocc = m->nocc, NN = N * N, i, j, k, it = 0;
    double a0 = (xc == XC_HF) ? 1.0 : 0.20;
    double *S = malloc(sizeof(double) * NN), *T = malloc(sizeof(double) * NN), *Vn = malloc(sizeof(double) * NN);
    double *H = malloc(sizeof(double) * NN), *X = calloc(NN, sizeof(double)), *P = calloc(NN, sizeof(double));
    double *J = malloc(sizeof(double) * NN), *K = malloc(sizeof(double) * NN), *Vx = malloc(sizeof(double) * NN);
    double *F = malloc(sizeof(double) * NN), *t1 = malloc(sizeof(double) * NN), *t2 = malloc(sizeof(double) * NN);
    double *Cp = malloc(sizeof(double) * NN), *C = malloc(sizeof(double) * NN), *w = malloc(sizeof(double) * N);
    double *Fh = malloc(sizeof(double) * NN * diis_space), *Eh = malloc(sizeof(double) * NN * diis_space);
    double *Bm = malloc(sizeof(double) * diis_space * diis_space), *cv = malloc(sizeof(double) * (diis_space + 1));
    long G = orc_grid_size(m, nrad, nth, nph);
    double *grid = (xc == XC_HF) ? NULL : malloc(sizeof(double) * 4 * G);
    double *eri = malloc(sizeof(double) * orc_n_eri(m));
    double Enn = orc_enuc(m), Eprev = 0.0, E = 0.0, err = 0.0;
    int nh = 0, head = 0, st = ST_MAXITER, rc = 0;

    orc_int1e(m, S, T, Vn);
    for (i = 0; i < NN; i++) H[i] = T[i] + Vn[i];
    orc_eri(m, eri);
    if (grid) orc_grid(m, nrad, nth, nph, grid);

    /* Loewdin X = U s^-1/2 U^T */
    orc_eigh(N, S, w, Cp);
    if (w[0] < 1e-8) { rc = -1; st = ST_INVALID; goto done; }
    for (i = 0; i < N; i++)
        for (j = 0; j < N; j++) {
            double s = 0.0;
            for (k = 0; k < N; k++) s += Cp[i * N + k] / sqrt(w[k]) * Cp[j * N + k];
            X[i * N + j] = s;
        }
    /* initial density (the paper's "initialise C_1" leaves the choice open):
     * guess 0: diagonal superposition of neutral-atom ground-state
     * occupations (STO-3G: H 1s 1; C/N/O/F 1s 2, 2s 2, 2p (Z-4)/3 each;
     * 6-31G: the valence occupation split evenly over the inner and outer
     * shells), scaled to N_e, used as rho_1 directly;  guess 1: core Hamiltonian -- diagonalise
     * X^T H X at iteration 0. */
    memcpy(F, H, sizeof(double) * NN);
    it = 0;
    if (guess == 0) {
        double tot = 0.0;
        for (i = 0; i < m->nshell; i++) {
            const oshell *s = &m->sh[i];
            int c;
            for (c = 0; c < (s->L ? 3 : 1); c++) P[(s->bf0 + c) * N + s->bf0 + c] = s->occ;
        }
        for (i = 0; i < N; i++) tot += P[i * N + i];
        for (i = 0; i < N; i++) P[i * N + i] *= m->nelec / tot;
        it = 1;
    }
    for (; it <= max_iter; it++) {
        if (it > 0) {
            ksum e1 = {0, 0}, e2 = {0, 0}, e3 = {0, 0};
            double exc = 0.0;
            orc_jk(m, eri, P, J, K);
            if (grid) exc = orc_xc(m, xc, G, grid, P, Vx); else memset(Vx, 0, sizeof(double) * NN);
            for (i = 0; i < NN; i++) F[i] = H[i] + J[i] - 0.5 * a0 * K[i] + Vx[i];
            for (i = 0; i < NN; i++) {
                ksum_add(&e1, P[i] * H[i]);
                ksum_add(&e2, 0.5 * P[i] * J[i]);
                ksum_add(&e3, -0.25 * a0 * P[i] * K[i]);
            }
            E = ksum_get(&e1) + ksum_get(&e2) + ksum_get(&e3) + exc + Enn;
            if (Eterms) {
                Eterms[0] = ksum_get(&e1); Eterms[1] = ksum_get(&e2); Eterms[2] = ksum_get(&e3);
                Eterms[3] = exc; Eterms[4] = Enn; Eterms[5] = E;
            }
            if (!isfinite(E)) { st = ST_DIVERGED; break; }
            /* e = X^T (F P S - S P F) X */
            matmul(N, F, 0, P, 0, t1);
            matmul(N, t1, 0, S, 0, t2);            /* FPS */
            for (i = 0; i < N; i++)
                for (j = 0; j < N; j++) t1[i * N + j] = t2[i * N + j] - t2[j * N + i];
            matmul(N, X, 1, t1, 0, t2);
            matmul(N, t2, 0, X, 0, t1);            /* e */
            err = 0.0;
            for (i = 0; i < NN; i++) if (fabs(t1[i]) > err) err = fabs(t1[i]);
            if (it > 1 && fabs(E - Eprev) < e_tol && err < comm_tol) { st = ST_CONVERGED; break; }
            if (it == max_iter) break;
            Eprev = E;
            /* DIIS: ring buffer of the last diis_space pairs */
            memcpy(Fh + (long)head * NN, F, sizeof(double) * NN);
            memcpy(Eh + (long)head * NN, t1, sizeof(double) * NN);
            head = (head + 1) % diis_space;
            if (nh < diis_space) nh++;
            {
                int n = nh, ok = 0, oldest;
                while (!ok && n > 0) {
                    /* slots of the n newest vectors, oldest first */
                    int sl[64];
                    for (i = 0; i < n; i++) sl[i] = ((head - n + i) % diis_space + diis_space) % diis_space;
                    for (i = 0; i < n; i++)
                        for (j = 0; j < n; j++) {
                            ksum b = {0, 0};
                            for (k = 0; k < NN; k++) ksum_add(&b, Eh[(long)sl[i] * NN + k] * Eh[(long)sl[j] * NN + k]);
                            Bm[i * n + j] = ksum_get(&b);
                        }
                    ok = diis_solve(n, Bm, cv);
                    if (ok) {
                        memset(F, 0, sizeof(double) * NN);
                        for (i = 0; i < n; i++)
                            for (k = 0; k < NN; k++) F[k] += cv[i] * Fh[(long)sl[i] * NN + k];
                    } else {
                        n--;
                    }
                }
                oldest = nh - n;
                nh -= oldest;                      /* dropped vectors leave the history */
            }
        }
        /* diagonalise X^T F X, C = X C', P = 2 C_occ C_occ^T */
        matmul(N, X, 1, F, 0, t1);
        matmul(N, t1, 0, X, 0, t2);
        orc_eigh(N, t2, w, Cp);
        matmul(N, X, 0, Cp, 0, C);
        for (i = 0; i < N; i++)
            for (j = 0; j < N; j++) {
                double s = 0.0;
                for (k = 0; k < nocc; k++) s += C[i * N + k] * C[j * N + k];
                P[i * N + j] = 2.0 * s;
            }
    }
    /* final orbital energies from the un-extrapolated F_k */
    matmul(N, X, 1, F, 0, t1);
    matmul(N, t1, 0, X, 0, t2);
    orc_eigh(N, t2, w, Cp);
    if (st == ST_MAXITER && it > max_iter) it = max_iter;
done:
    *E_out = E;
    if (eps) memcpy(eps, w, sizeof(double) * N);
    if (P_out) memcpy(P_out, P, sizeof(double) * NN);
    *niter = it;
    *status = st;
    free(S); free(T); free(Vn); free(H); free(X); free(P); free(J); free(K); free(Vx); free(F);
    free(t1); free(t2); free(Cp); free(C); free(w); free(Fh); free(Eh); free(Bm); free(cv);
    free(grid); free(eri);
    return rc;
}
