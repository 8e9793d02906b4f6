/*
 * clb3d_oracle.c -- plain FP64 CPU oracle for the three-dimensional form of the central-moment
 * lattice Boltzmann (CLB) method for incompressible thermal flow (Fei, Luo, Lin, Li;
 * arXiv 1710.10569).  The paper derives and tests the method in two dimensions and states in its
 * conclusions (Sec. 4) that it extends directly to three; this file takes every two-dimensional
 * definition dimension by dimension.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  This is the slow, obviously correct reference that the
 * GPU library's 3D path is checked against.  It shares no code, header, table or helper with the
 * GPU library (nor with the two-dimensional oracle).  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it.
 *
 * What it computes, following Secs. 2.1-2.2 with a third coordinate:
 *   Flow, D3Q27: the velocity set {0, +1, -1}^3 (the three-dimensional product of the set behind
 *     Eq. 4); raw moments k_abc = sum_i f_i e_ix^a e_iy^b e_iz^c and central moments
 *     k~_abc = sum_i f_i (e_ix - u_x)^a (e_iy - u_y)^b (e_iz - u_z)^c for a, b, c in {0, 1, 2}
 *     (Eq. 5); Gamma = M f (Eq. 7a) and Gamma~ = N(u) Gamma (Eq. 7b), with N(u) the binomial
 *     expansion of (e - u)^a written out entry by entry; the collision of Eq. 8,
 *     Gamma~* = (I - S) Gamma~ + S Gamma~^eq + (I - S/2) C; f* = M^-1 N^-1 Gamma~*; streaming
 *     (Eq. 12); rho and u of Eq. 13.
 *   Temperature, D3Q7: rest and the six axis vectors; moments [k000, k100, k010, k001, k200,
 *     k020, k002] (Eq. 15), N_T(u) the same binomial expansion (Eq. 18), the collision of Eq. 19,
 *     streaming (Eq. 22), T of Eq. 23.
 *   Eq. 3 with gravity along -z: F = (F_vx, F_vy, F_vz + g beta (T - T0)).
 *
 * Readings (each one is listed with its reason in the design notes of the repository):
 *   - Equilibrium central moments: Gamma~^eq_abc = rho m(a) m(b) m(c) with m(0) = 1, m(1) = 0,
 *     m(2) = c_s^2 = 1/3 -- the pattern of Eq. 9 (k~20 = k~02 = rho c_s^2, k~22 = rho c_s^4, odd
 *     orders zero).  The equilibrium populations are then the product rho psi(e_x, u_x)
 *     psi(e_y, u_y) psi(e_z, u_z) of the one-dimensional factors of the D2Q9 equilibrium.
 *   - Forcing: C_abc = sum_d F_d [a_d = 1] prod_{d' != d} m(a_d') -- the pattern of Eq. 11
 *     (C_10 = F_x, C_21 = c_s^2 F_y, C_12 = c_s^2 F_x, all other entries zero).
 *   - Relaxation S: conserved moments (orders 0 and 1) 0; the three diagonal second-order moments
 *     relax their trace with s_b and their deviatoric part with s_nu (block s_nu I + (s_b - s_nu)/3
 *     J, the three-dimensional form of Eq. 8's [[s+, s-], [s-, s+]] block); k~110, k~101, k~011
 *     with s_nu; third order (k~210, k~201, k~120, k~021, k~102, k~012, k~111) s3; fourth order
 *     (k~220, k~202, k~022, k~211, k~121, k~112) s4; fifth order (k~221, k~212, k~122) s5; sixth
 *     order (k~222) s6.  s_b and s3..s6 default to 1, as the paper's tunable rates do (Sec. 3).
 *   - D3Q7: weights 1/4 (rest) and 1/8, so c_{T,s}^2 = 1/4 and alpha = (1/lambda1 - 1/2)/4, as in
 *     two dimensions; Gamma~_T^eq = [T, 0, 0, 0, T/4, T/4, T/4]; S_T = diag(1, l1, l1, l1, l2, l2, l2).
 *   - Domain: periodic in x and y; in z periodic or bounded by walls on the nodes z = 0 (bottom)
 *     and z = nz - 1 (top), H = nz - 1.  Walls move tangentially (u_w,z = 0) and hold a Dirichlet
 *     temperature or are adiabatic (T_b = (4 T(x_f) - T(x_ff)) / 3, as in two dimensions).
 *   - Wall closure.  The paper gives no three-dimensional wall scheme.  Both lattices use the
 *     non-equilibrium extrapolation that the paper uses for temperature walls (Guo et al.), with
 *     x_f = the inner neighbour along z and every population replaced:
 *         g_i = g^eq_i(T_b, u_w) + g_i(x_f) - g^eq_i(T_f, u_f),
 *         f_i = f^eq_i(rho_b, u_w - F_b/(2 rho_b)) + f_i(x_f) - f^eq_i(rho_f, u_f - F_f/(2 rho_f)),
 *     so that sum f = rho_b and Eq. 13 returns u_w at the wall.  The wall density is the node's
 *     mass balance, as in the two-dimensional wall reading: rho_b = the known populations after
 *     streaming + the populations the node sent out of the domain the step before, so a closed
 *     box neither gains nor loses mass.  The wall temperature enters F_b.
 *
 * Pinned by (tests): the closed forms of both equilibria, the definition of central moments, exact
 * conservation, the two-dimensional oracle on a periodic slab one node thick (s_b = s_nu there),
 * symmetry under a cyclic relabelling of the axes, the exact decay of an ABC flow, shear and
 * temperature waves in a moving frame, sound attenuation at the bulk viscosity set by s_b, the
 * analytic Poiseuille and conduction states, the imposed wall values and exact mass conservation
 * in a closed box.  Parity unpinned: the rates s5 and s6 (they relax only the fifth- and
 * sixth-order moments k~221, k~212, k~122 and k~222, which no pinned flow excites measurably), and
 * the wall closure's choice of replacing every population rather than only the unknown ones (held
 * only by its invariants: the imposed wall velocity and temperature, second-order Poiseuille, exact
 * mass conservation and the conduction state).
 *
 * State convention, as in two dimensions: f[27][n] and g[7][n] hold the populations of time t
 * after streaming and before the wall step; unknown entries (sources beyond a wall) are NaN.  Node
 * (x, y, z) has index (z ny + y) nx + x.  out[27][n] holds the populations f*_k that wall nodes
 * sent out of the domain in the last step (entry k of a node is defined where x + e_k lies beyond
 * a wall).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define CS2 (1.0 / 3.0)   /* c_s^2 of the flow lattice */
#define CT2 (1.0 / 4.0)   /* c_{T,s}^2 of the temperature lattice */

enum { Z_PERIODIC = 0, Z_DIRICHLET = 1, Z_ADIABATIC = 2 };

/* D3Q27: rest; the six axis vectors; the twelve edge vectors; the eight corner vectors.  The first
 * seven are the D3Q7 set.  Opposite vectors sit next to each other (1-2, 3-4, ...). */
static const int EX[27] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1};
static const int EY[27] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, -1, 1, 1, -1};
static const int EZ[27] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1, 1, -1, -1, 1, 1, -1, 1, -1};

/* Moment order (a, b, c) of Gamma, by total order: the 3D form of Eq. 6's ordering. */
static const int MA[27][3] = {
    {0, 0, 0},
    {1, 0, 0}, {0, 1, 0}, {0, 0, 1},
    {2, 0, 0}, {0, 2, 0}, {0, 0, 2}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1},
    {2, 1, 0}, {2, 0, 1}, {1, 2, 0}, {0, 2, 1}, {1, 0, 2}, {0, 1, 2}, {1, 1, 1},
    {2, 2, 0}, {2, 0, 2}, {0, 2, 2}, {2, 1, 1}, {1, 2, 1}, {1, 1, 2},
    {2, 2, 1}, {2, 1, 2}, {1, 2, 2},
    {2, 2, 2},
};
/* D3Q7 moment order: [k000, k100, k010, k001, k200, k020, k002]. */
static const int MT[7][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {2, 0, 0}, {0, 2, 0}, {0, 0, 2}};

typedef struct {
    int nx, ny, nz;
    int zkind[2];        /* bottom (z = 0), top (z = nz - 1): periodic / Dirichlet / adiabatic */
    double uw[2][2];     /* tangential wall velocity (x, y) of bottom and top */
    double Tw[2];        /* wall temperature (Dirichlet) */
    double T0;           /* reference temperature of Eq. 3 */
    double s_nu, s_b, s3, s4, s5, s6;
    double lam1, lam2;
    double g_beta, Fv[3];
    double *f, *g, *fn, *gn, *out;
    double M[27 * 27], Minv[27 * 27], MTm[49], MTinv[49];
    int opp[27];
    int bad;
} orc3_lattice;

/* ------------------------------------------------------------------------------------------ */
/* Small dense linear algebra (plain loops).                                                   */

static void matvec(int n, const double* A, const double* x, double* y)
{
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int j = 0; j < n; ++j) s += A[i * n + j] * x[j];
        y[i] = s;
    }
}

/* Gauss-Jordan inversion with partial pivoting; returns 0 on success. */
static int invert(int n, const double* A, double* Ainv)
{
    double* a = (double*)malloc((size_t)n * 2 * n * sizeof(double));
    if (!a) return -1;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < 2 * n; ++j) a[i * 2 * n + j] = j < n ? A[i * n + j] : (j - n == i ? 1.0 : 0.0);
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(a[r * 2 * n + c]) > fabs(a[p * 2 * n + c])) p = r;
        if (a[p * 2 * n + c] == 0.0) { free(a); return -1; }
        if (p != c)
            for (int j = 0; j < 2 * n; ++j) { double t = a[c * 2 * n + j]; a[c * 2 * n + j] = a[p * 2 * n + j]; a[p * 2 * n + j] = t; }
        const double d = a[c * 2 * n + c];
        for (int j = 0; j < 2 * n; ++j) a[c * 2 * n + j] /= d;
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const double m = a[r * 2 * n + c];
            if (m != 0.0)
                for (int j = 0; j < 2 * n; ++j) a[r * 2 * n + j] -= m * a[c * 2 * n + j];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Ainv[i * n + j] = a[i * 2 * n + n + j];
    free(a);
    return 0;
}

/* Solve L x = b for a unit lower-triangular L (forward substitution): N and N_T are unit lower
 * triangular because the moments are ordered by total order. */
static void solve_unit_lower(int n, const double* L, const double* b, double* x)
{
    for (int i = 0; i < n; ++i) {
        double s = b[i];
        for (int j = 0; j < i; ++j) s -= L[i * n + j] * x[j];
        x[i] = s;
    }
}

static double ipow(double v, int p)
{
    double r = 1.0;
    for (int k = 0; k < p; ++k) r *= v;
    return r;
}

static double binom(int a, int p) { return (a == 2 && p == 1) ? 2.0 : 1.0; }   /* a, p in {0, 1, 2}, p <= a */

/* ------------------------------------------------------------------------------------------ */
/* Transforms.                                                                                  */

/* Eq. 7a: M[m][i] = e_ix^a e_iy^b e_iz^c for the m-th moment (a, b, c) of ord. */
static void build_M(int nm, const int (*ord)[3], double* M)
{
    for (int m = 0; m < nm; ++m)
        for (int i = 0; i < nm; ++i)
            M[m * nm + i] = ipow(EX[i], ord[m][0]) * ipow(EY[i], ord[m][1]) * ipow(EZ[i], ord[m][2]);
}

/* Eq. 7b: (e - u)^a = sum_{p <= a} C(a, p) e^p (-u)^(a - p) in each coordinate, so
 * N[m][q] = prod_d C(a_d, p_d) (-u_d)^(a_d - p_d) where p <= a componentwise, else 0. */
static void build_N(int nm, const int (*ord)[3], const double u[3], double* N)
{
    for (int m = 0; m < nm; ++m)
        for (int q = 0; q < nm; ++q) {
            double v = 1.0;
            for (int d = 0; d < 3; ++d) {
                const int a = ord[m][d], p = ord[q][d];
                if (p > a) { v = 0.0; break; }
                v *= binom(a, p) * ipow(-u[d], a - p);
            }
            N[m * nm + q] = v;
        }
}

static double m_eq(int a) { return a == 0 ? 1.0 : (a == 1 ? 0.0 : CS2); }

/* Equilibrium central moments (Eq. 9's pattern) and forcing central moments (Eq. 11's pattern). */
static void gamma_eq(double rho, double* G)
{
    for (int m = 0; m < 27; ++m) G[m] = rho * m_eq(MA[m][0]) * m_eq(MA[m][1]) * m_eq(MA[m][2]);
}

static void forcing(const double F[3], double* C)
{
    for (int m = 0; m < 27; ++m) {
        double c = 0.0;
        for (int d = 0; d < 3; ++d) {
            if (MA[m][d] != 1) continue;
            double p = F[d];
            for (int e = 0; e < 3; ++e)
                if (e != d) p *= m_eq(MA[m][e]);
            c += p;
        }
        C[m] = c;
    }
}

/* Relaxation matrix S (see the header). */
static void build_S(const orc3_lattice* L, double* S)
{
    memset(S, 0, 27 * 27 * sizeof(double));
    for (int m = 0; m < 27; ++m) {
        const int a = MA[m][0], b = MA[m][1], c = MA[m][2], o = a + b + c;
        double s = 0.0;
        if (o == 2 && (a == 1 || b == 1 || c == 1)) s = L->s_nu;   /* k~110, k~101, k~011 */
        else if (o == 3) s = L->s3;
        else if (o == 4) s = L->s4;
        else if (o == 5) s = L->s5;
        else if (o == 6) s = L->s6;
        S[m * 27 + m] = s;
    }
    /* diagonal second-order block, moments 4, 5, 6 */
    for (int i = 4; i < 7; ++i)
        for (int j = 4; j < 7; ++j)
            S[i * 27 + j] = (i == j ? L->s_nu : 0.0) + (L->s_b - L->s_nu) / 3.0;
}

/* f^eq: the populations whose central moments are Gamma~^eq, f^eq = M^-1 N(u)^-1 Gamma~^eq. */
static void feq27(const orc3_lattice* L, double rho, const double u[3], double* out)
{
    double G[27], N[27 * 27], R[27];
    gamma_eq(rho, G);
    build_N(27, MA, u, N);
    solve_unit_lower(27, N, G, R);
    matvec(27, L->Minv, R, out);
}

static void geq7(const orc3_lattice* L, double T, const double u[3], double* out)
{
    const double G[7] = {T, 0, 0, 0, T * CT2, T * CT2, T * CT2};
    double N[49], R[7];
    build_N(7, MT, u, N);
    solve_unit_lower(7, N, G, R);
    matvec(7, L->MTinv, R, out);
}

/* Eq. 8 for one node. */
static void collide27(const orc3_lattice* L, const double* f, double rho, const double u[3], const double F[3],
                      double* fpost)
{
    double G[27], Gt[27], Gs[27], R[27], Geq[27], C[27], N[27 * 27], S[27 * 27];
    gamma_eq(rho, Geq);
    forcing(F, C);
    matvec(27, L->M, f, G);
    build_N(27, MA, u, N);
    matvec(27, N, G, Gt);
    build_S(L, S);
    for (int i = 0; i < 27; ++i) {
        double s = 0.0;
        for (int j = 0; j < 27; ++j) {
            const double I = (i == j) ? 1.0 : 0.0;
            s += (I - S[i * 27 + j]) * Gt[j] + S[i * 27 + j] * Geq[j] + (I - 0.5 * S[i * 27 + j]) * C[j];
        }
        Gs[i] = s;
    }
    solve_unit_lower(27, N, Gs, R);
    matvec(27, L->Minv, R, fpost);
}

/* Eq. 19 for one node. */
static void collide7(const orc3_lattice* L, const double* g, double T, const double u[3], double* gpost)
{
    double N[49], G[7], Gt[7], Gs[7], R[7];
    const double Geq[7] = {T, 0, 0, 0, T * CT2, T * CT2, T * CT2};
    const double ST[7] = {1.0, L->lam1, L->lam1, L->lam1, L->lam2, L->lam2, L->lam2};
    matvec(7, L->MTm, g, G);
    build_N(7, MT, u, N);
    matvec(7, N, G, Gt);
    for (int i = 0; i < 7; ++i) Gs[i] = (1.0 - ST[i]) * Gt[i] + ST[i] * Geq[i];
    solve_unit_lower(7, N, Gs, R);
    matvec(7, L->MTinv, R, gpost);
}

/* ------------------------------------------------------------------------------------------ */
/* Macroscopic quantities: Eq. 23 (T), Eq. 3 (F, gravity along -z), Eq. 13 (rho, u).            */

static void macro_of(const orc3_lattice* L, const double* f, const double* g, double* rho, double u[3],
                     double* T, double F[3])
{
    double t = 0.0;
    for (int i = 0; i < 7; ++i) t += g[i];
    *T = t;
    F[0] = L->Fv[0];
    F[1] = L->Fv[1];
    F[2] = L->Fv[2] + L->g_beta * (t - L->T0);
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < 27; ++i) {
        r += f[i];
        j[0] += f[i] * EX[i];
        j[1] += f[i] * EY[i];
        j[2] += f[i] * EZ[i];
    }
    *rho = r;
    for (int d = 0; d < 3; ++d) u[d] = (j[d] + 0.5 * F[d]) / r;
}

/* ------------------------------------------------------------------------------------------ */
/* Wall step.                                                                                   */

static size_t idx3(const orc3_lattice* L, int x, int y, int z) { return ((size_t)z * L->ny + y) * L->nx + x; }

static void load_node(const orc3_lattice* L, size_t k, double* f, double* g)
{
    const size_t n = (size_t)L->nx * L->ny * L->nz;
    for (int i = 0; i < 27; ++i) f[i] = L->f[i * n + k];
    for (int i = 0; i < 7; ++i) g[i] = L->g[i * n + k];
}

/* Wall step at node (x, y, z) on the bottom (w = 0) or top (w = 1) wall: f, g hold the node's
 * state(t) on entry and the reconstructed populations on exit. */
static void wall_step(const orc3_lattice* L, int x, int y, int z, int w, double* f, double* g)
{
    const size_t n = (size_t)L->nx * L->ny * L->nz, k = idx3(L, x, y, z);
    const int dz = w == 0 ? 1 : -1;            /* inward normal */
    double ff[27], gf[7], rf, uf[3], Tf, Ff[3];
    load_node(L, idx3(L, x, y, z + dz), ff, gf);
    macro_of(L, ff, gf, &rf, uf, &Tf, Ff);
    double Tb;
    if (L->zkind[w] == Z_DIRICHLET) {
        Tb = L->Tw[w];
    } else {
        double fff[27], gff[7], rff, uff[3], Tff, Fff[3];
        load_node(L, idx3(L, x, y, z + 2 * dz), fff, gff);
        macro_of(L, fff, gff, &rff, uff, &Tff, Fff);
        Tb = (4.0 * Tf - Tff) / 3.0;
    }
    const double uw[3] = {L->uw[w][0], L->uw[w][1], 0.0};
    /* temperature: non-equilibrium extrapolation of all seven populations */
    double ge_b[7], ge_f[7];
    geq7(L, Tb, uw, ge_b);
    geq7(L, Tf, uf, ge_f);
    for (int i = 0; i < 7; ++i) g[i] = ge_b[i] + gf[i] - ge_f[i];
    /* force from the wall temperature */
    const double Fb[3] = {L->Fv[0], L->Fv[1], L->Fv[2] + L->g_beta * (Tb - L->T0)};
    /* density: the node's mass balance (known populations + those it sent out the step before) */
    double rho_b = 0.0;
    for (int i = 0; i < 27; ++i) {
        const int unknown = EZ[i] * dz > 0;    /* source x - e_i beyond the wall */
        rho_b += unknown ? L->out[L->opp[i] * n + k] : f[i];
    }
    /* flow: non-equilibrium extrapolation of all 27 populations */
    const double vb[3] = {uw[0] - 0.5 * Fb[0] / rho_b, uw[1] - 0.5 * Fb[1] / rho_b, -0.5 * Fb[2] / rho_b};
    const double vf[3] = {uf[0] - 0.5 * Ff[0] / rf, uf[1] - 0.5 * Ff[1] / rf, uf[2] - 0.5 * Ff[2] / rf};
    double fe_b[27], fe_f[27];
    feq27(L, rho_b, vb, fe_b);
    feq27(L, rf, vf, fe_f);
    for (int i = 0; i < 27; ++i) f[i] = fe_b[i] + ff[i] - fe_f[i];
}

static int wall_of(const orc3_lattice* L, int z)
{
    if (L->zkind[0] == Z_PERIODIC) return -1;
    return z == 0 ? 0 : (z == L->nz - 1 ? 1 : -1);
}

/* Wall step + macroscopic step at one node. */
static void pre_collision(orc3_lattice* L, int x, int y, int z, double* f, double* g, double* rho, double u[3],
                          double* T, double F[3])
{
    const size_t k = idx3(L, x, y, z);
    load_node(L, k, f, g);
    const int w = wall_of(L, z);
    if (w >= 0) wall_step(L, x, y, z, w, f, g);
    for (int i = 0; i < 27; ++i)
        if (isnan(f[i])) L->bad = 1;
    for (int i = 0; i < 7; ++i)
        if (isnan(g[i])) L->bad = 1;
    macro_of(L, f, g, rho, u, T, F);
}

/* ------------------------------------------------------------------------------------------ */
/* Public C interface (loaded with ctypes by the tests).                                        */

void orc3_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* zkind: bottom and top kind (both periodic or both walls); uw: (ux, uy) of bottom then top;
 * Tw: bottom and top wall temperatures. */
orc3_lattice* orc3_create(int nx, int ny, int nz, const int* zkind, const double* uw, const double* Tw, double T0)
{
    if (nx < 1 || ny < 1 || nz < 1) return NULL;
    if ((zkind[0] == Z_PERIODIC) != (zkind[1] == Z_PERIODIC)) return NULL;
    if (zkind[0] != Z_PERIODIC && nz < 3) return NULL;
    orc3_lattice* L = (orc3_lattice*)calloc(1, sizeof(orc3_lattice));
    if (!L) return NULL;
    L->nx = nx; L->ny = ny; L->nz = nz;
    for (int w = 0; w < 2; ++w) {
        L->zkind[w] = zkind[w];
        L->uw[w][0] = uw[2 * w];
        L->uw[w][1] = uw[2 * w + 1];
        L->Tw[w] = Tw[w];
    }
    L->T0 = T0;
    L->s_nu = L->s_b = L->s3 = L->s4 = L->s5 = L->s6 = 1.0;
    L->lam1 = L->lam2 = 1.0;
    for (int i = 0; i < 27; ++i)
        for (int j = 0; j < 27; ++j)
            if (EX[j] == -EX[i] && EY[j] == -EY[i] && EZ[j] == -EZ[i]) L->opp[i] = j;
    build_M(27, MA, L->M);
    build_M(7, MT, L->MTm);
    const size_t n = (size_t)nx * ny * nz;
    L->f = (double*)malloc(27 * n * sizeof(double));
    L->fn = (double*)malloc(27 * n * sizeof(double));
    L->g = (double*)malloc(7 * n * sizeof(double));
    L->gn = (double*)malloc(7 * n * sizeof(double));
    L->out = (double*)malloc(27 * n * sizeof(double));
    if (!L->f || !L->fn || !L->g || !L->gn || !L->out || invert(27, L->M, L->Minv) || invert(7, L->MTm, L->MTinv)) {
        free(L->f); free(L->fn); free(L->g); free(L->gn); free(L->out); free(L);
        return NULL;
    }
    for (size_t i = 0; i < 27 * n; ++i) L->f[i] = L->out[i] = NAN;
    for (size_t i = 0; i < 7 * n; ++i) L->g[i] = NAN;
    return L;
}

void orc3_destroy(orc3_lattice* L)
{
    if (!L) return;
    free(L->f); free(L->fn); free(L->g); free(L->gn); free(L->out);
    free(L);
}

/* tau_nu = 1/s_nu (nu = (tau_nu - 1/2)/3); tau_alpha = 1/lambda1 (alpha = (tau_alpha - 1/2)/4). */
void orc3_set_params(orc3_lattice* L, double tau_nu, double tau_alpha, double g_beta)
{
    L->s_nu = 1.0 / tau_nu;
    L->lam1 = 1.0 / tau_alpha;
    L->g_beta = g_beta;
}

void orc3_set_relaxation(orc3_lattice* L, double s_b, double s3, double s4, double s5, double s6, double lam2)
{
    L->s_b = s_b; L->s3 = s3; L->s4 = s4; L->s5 = s5; L->s6 = s6; L->lam2 = lam2;
}

void orc3_set_body_force(orc3_lattice* L, double Fx, double Fy, double Fz)
{
    L->Fv[0] = Fx; L->Fv[1] = Fy; L->Fv[2] = Fz;
}

/* Initial state: g = g^eq(T, u0), f = f^eq(rho0, u0 - F/(2 rho0)) with F from T, so that Eq. 13
 * returns (rho0, u0) and Eq. 23 returns T; NULL arrays mean rho = 1, u = 0, T = T0.  The outgoing
 * populations of the step before t = 0 are the initial values of the unknown populations they
 * pair with, out[opp(i)] = f_i, so that a wall node's mass balance returns rho0.  u is given as
 * three planes (x, y, z) of n values. */
void orc3_init(orc3_lattice* L, const double* rho, const double* u, const double* T)
{
    const size_t n = (size_t)L->nx * L->ny * L->nz;
    for (size_t k = 0; k < n; ++k) {
        const double r = rho ? rho[k] : 1.0;
        const double t = T ? T[k] : L->T0;
        const double u0[3] = {u ? u[k] : 0.0, u ? u[n + k] : 0.0, u ? u[2 * n + k] : 0.0};
        const double F[3] = {L->Fv[0], L->Fv[1], L->Fv[2] + L->g_beta * (t - L->T0)};
        const double v[3] = {u0[0] - 0.5 * F[0] / r, u0[1] - 0.5 * F[1] / r, u0[2] - 0.5 * F[2] / r};
        double fe[27], ge[7];
        feq27(L, r, v, fe);
        geq7(L, t, u0, ge);
        for (int i = 0; i < 27; ++i) L->f[i * n + k] = fe[i];
        for (int i = 0; i < 7; ++i) L->g[i * n + k] = ge[i];
        for (int i = 0; i < 27; ++i) L->out[L->opp[i] * n + k] = fe[i];
    }
    L->bad = 0;
}

/* n time steps (wall step -> macroscopic -> collision -> streaming).  Returns 0, or -1 if a
 * population that should have been reconstructed by the wall step was still unknown. */
int orc3_step(orc3_lattice* L, long long nsteps)
{
    const int nx = L->nx, ny = L->ny, nz = L->nz;
    const size_t n = (size_t)nx * ny * nz;
    for (long long s = 0; s < nsteps; ++s) {
        for (size_t i = 0; i < 27 * n; ++i) L->fn[i] = NAN;
        for (size_t i = 0; i < 7 * n; ++i) L->gn[i] = NAN;
#pragma omp parallel for schedule(static) collapse(2)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    double f[27], g[7], fp[27], gp[7], rho, u[3], T, F[3];
                    pre_collision(L, x, y, z, f, g, &rho, u, &T, F);
                    collide27(L, f, rho, u, F, fp);
                    collide7(L, g, T, u, gp);
                    /* Eqs. 12 and 22: f_i(x + e_i, t + 1) = f_i*(x, t); targets beyond a wall are
                     * kept as the node's outgoing populations. */
                    const size_t k = idx3(L, x, y, z);
                    for (int i = 0; i < 27; ++i) {
                        const int tx = (x + EX[i] + nx) % nx, ty = (y + EY[i] + ny) % ny;
                        int tz = z + EZ[i];
                        if (L->zkind[0] == Z_PERIODIC) tz = (tz + nz) % nz;
                        if (tz < 0 || tz >= nz) {
                            L->out[i * n + k] = fp[i];
                            continue;
                        }
                        const size_t t = idx3(L, tx, ty, tz);
                        L->fn[i * n + t] = fp[i];
                        if (i < 7) L->gn[i * n + t] = gp[i];
                    }
                }
        double* tmp = L->f; L->f = L->fn; L->fn = tmp;
        tmp = L->g; L->g = L->gn; L->gn = tmp;
    }
    return L->bad ? -1 : 0;
}

/* rho, u (three planes), T of the current time: the wall step and Eqs. 3, 13, 23 on state(t). */
int orc3_moments(orc3_lattice* L, double* rho, double* u, double* T)
{
    const int nx = L->nx, ny = L->ny, nz = L->nz;
    const size_t n = (size_t)nx * ny * nz;
#pragma omp parallel for schedule(static) collapse(2)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                double f[27], g[7], r, v[3], t, F[3];
                pre_collision(L, x, y, z, f, g, &r, v, &t, F);
                const size_t k = idx3(L, x, y, z);
                if (rho) rho[k] = r;
                if (u) { u[k] = v[0]; u[n + k] = v[1]; u[2 * n + k] = v[2]; }
                if (T) T[k] = t;
            }
    return L->bad ? -1 : 0;
}

/* Copy out / in state(t): f as [27][nz][ny][nx], g as [7][nz][ny][nx]. */
void orc3_get_state(const orc3_lattice* L, double* f, double* g)
{
    const size_t n = (size_t)L->nx * L->ny * L->nz;
    if (f) memcpy(f, L->f, 27 * n * sizeof(double));
    if (g) memcpy(g, L->g, 7 * n * sizeof(double));
}

void orc3_set_state(orc3_lattice* L, const double* f, const double* g)
{
    const size_t n = (size_t)L->nx * L->ny * L->nz;
    if (f) memcpy(L->f, f, 27 * n * sizeof(double));
    if (g) memcpy(L->g, g, 7 * n * sizeof(double));
    L->bad = 0;
}

void orc3_get_outgoing(const orc3_lattice* L, double* out)
{
    memcpy(out, L->out, 27 * (size_t)L->nx * L->ny * L->nz * sizeof(double));
}

/* ---- single-node access for the algebra tests ---- */
void orc3_velocities(int* ex, int* ey, int* ez)
{
    memcpy(ex, EX, sizeof EX); memcpy(ey, EY, sizeof EY); memcpy(ez, EZ, sizeof EZ);
}
void orc3_moment_order(int* ord) { memcpy(ord, MA, sizeof MA); }
void orc3_matrix_M(const orc3_lattice* L, double* out) { memcpy(out, L->M, sizeof L->M); }
void orc3_matrix_N(double ux, double uy, double uz, double* out)
{
    const double u[3] = {ux, uy, uz};
    build_N(27, MA, u, out);
}
void orc3_matrix_S(const orc3_lattice* L, double* out) { build_S(L, out); }
void orc3_feq(const orc3_lattice* L, double rho, double ux, double uy, double uz, double* out)
{
    const double u[3] = {ux, uy, uz};
    feq27(L, rho, u, out);
}
void orc3_geq(const orc3_lattice* L, double T, double ux, double uy, double uz, double* out)
{
    const double u[3] = {ux, uy, uz};
    geq7(L, T, u, out);
}
/* Collision of one node given its pre-collision f and the force: rho, u from Eq. 13. */
void orc3_collide27(const orc3_lattice* L, const double* f, double Fx, double Fy, double Fz, double* out)
{
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < 27; ++i) { r += f[i]; j[0] += f[i] * EX[i]; j[1] += f[i] * EY[i]; j[2] += f[i] * EZ[i]; }
    const double F[3] = {Fx, Fy, Fz};
    const double u[3] = {(j[0] + 0.5 * Fx) / r, (j[1] + 0.5 * Fy) / r, (j[2] + 0.5 * Fz) / r};
    collide27(L, f, r, u, F, out);
}
void orc3_collide7(const orc3_lattice* L, const double* g, double ux, double uy, double uz, double* out)
{
    double T = 0.0;
    for (int i = 0; i < 7; ++i) T += g[i];
    const double u[3] = {ux, uy, uz};
    collide7(L, g, T, u, out);
}
