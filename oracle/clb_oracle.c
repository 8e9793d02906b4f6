/*
 * clb_oracle.c -- plain FP64 CPU oracle for the central-moment lattice Boltzmann (CLB) method for
 * incompressible thermal flow (Fei, Luo, Lin, Li; arXiv 1710.10569).
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  This is the slow, obviously correct reference that the
 * GPU library is checked against.  It shares no code, header, table or helper with the GPU
 * library.  Only the test suite, the smoke check and the CPU-baseline leg of the benchmark load it.
 *
 * What it computes, in the paper's order and notation:
 *   Sec. 2.1  D2Q9 CLB for the flow: velocity set (Eq. 4), raw moments Gamma = M f (Eqs. 5-7a),
 *             central moments Gamma~ = N(u) Gamma (Eq. 7b), collision (Eq. 8) with the relaxation
 *             matrix S, the equilibrium central moments (Eq. 9) and the consistent forcing term
 *             C (Eq. 11), back-transform f* = M^-1 N^-1 Gamma~* and streaming (Eq. 12), and the
 *             macroscopic density and velocity (Eq. 13).
 *   Sec. 2.2  D2Q5 CLB for temperature: M_T (Eq. 17), N_T (Eq. 18), collision (Eq. 19) to the
 *             equilibrium of Eq. 20, back-transform (Eq. 21), streaming (Eq. 22), T (Eq. 23).
 *   Eq. 3     Boussinesq coupling F = -g beta (T - T0) + F_v with gravity along -y.
 *   Sec. 3    wall conditions: non-equilibrium bounce-back (Zou-He) for the flow populations and
 *             non-equilibrium extrapolation (Guo et al.) for the temperature populations.
 *
 * Readings where the paper is silent or misprinted (each one is listed with its reason in the
 * design notes of the repository):
 *   - Eq. 7b row k~02: the entry multiplying k01 is -2 u_y (the printed +2 u_y contradicts the
 *     definition of Eq. 5b; N_T of Eq. 18 carries the correct sign).
 *   - The bulk rate s_b and the high-order rates s3, s4, lambda2 default to 1.0 (Sec. 3 sets the
 *     tunable high-order rates to 1.0 and gives no other value for s_b).
 *   - c_{T,s}^2 = 1/4 (Sec. 3 default c_sT = 1/2), so alpha = (1/lambda1 - 1/2)/4.
 *   - F is a force density with rho0 = 1; F enters u through Eq. 13 and is evaluated from the
 *     temperature of the same pre-collision state.
 *   - Walls sit on nodes.  A population is unknown at a wall node when its streaming source lies
 *     outside the domain; those are marked NaN in the state and must be replaced by the wall step.
 *   - Wall step order at a wall node: temperature NEE first (all five g), then the force from the
 *     wall temperature, then the flow: force-corrected Zou-He on edges, non-equilibrium bounce-back
 *     of the opposite pairs at corners.
 *   - Density of a wall node.  Zou-He's own density (from the normal momentum constraint) does not
 *     conserve mass: along a wall the nodes exchange mass with the fluid, and in a closed buoyant
 *     cavity the corners and edges leave a net loss at every step, so no steady state exists.  A
 *     wall node whose wall is impermeable (u_w.n = 0; every corner) therefore takes as its density
 *     the mass it holds after streaming plus the mass it sent out of the domain the step before,
 *     rho_b = sum_known f_i(t) + sum_k f*_k(t-1) (k: directions leaving the domain), so the node
 *     exchanges no mass with the outside.  The unknown populations still satisfy Zou-He's
 *     constraints (sum f e = rho_b u_w - F/2, so Eq. 13 returns u_w) and the rest population f_0
 *     takes up the difference, f_0 = rho_b - sum_{i>0} f_i.  For a stationary wall the unknowns do
 *     not depend on rho_b, so only f_0 differs from plain Zou-He.  Permeable walls keep Zou-He's
 *     density: mass flows through them.
 *   - Adiabatic walls: T_b = (4 T(x_f) - T(x_ff)) / 3 (second-order zero normal gradient).
 *   - Corners: the inner neighbour is the diagonal one; for temperature a Dirichlet wall wins over
 *     an adiabatic one, and between two walls of the same kind the west/east wall's data is used;
 *     the corner's wall velocity is the west/east wall's.
 *
 * Parity unpinned: no printed value, closed form or invariant fixes these choices, so they hold only
 * as readings, shared by construction with the GPU library: the default s_b = 1, the corner data
 * (which wall's velocity and temperature a corner takes, the diagonal temperature extrapolation and
 * the split of a corner's unknowns) and the wall velocity of the temperature-only mode.  The wall
 * density is pinned by exact mass conservation in closed domains and by the steady state it allows.
 *
 * State convention: the arrays f[9][n] and g[5][n] hold the populations of time t after streaming
 * and before the wall step ("state(t)").  One step = wall step -> macroscopic -> collision ->
 * streaming (push) -> state(t+1).  Node (x, y) has index y*nx + x.  The array out[9][n] holds the
 * flow populations f*_k that wall nodes sent out of the domain in the last step (entry k of node x
 * defined where x + e_k lies beyond a wall); it is part of the state.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- Eq. 4: the D2Q9 velocity set; its first five vectors are the D2Q5 set (Sec. 2.2) ---- */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};   /* e_OPP[i] = -e_i */

#define CS2 (1.0 / 3.0)   /* c_s^2 of the D2Q9 lattice (after Eq. 9) */
#define CT2 (1.0 / 4.0)   /* c_{T,s}^2 of the D2Q5 lattice (Sec. 3 default c_sT = 1/2) */

enum { W_PERIODIC = 0, W_DIRICHLET = 1, W_ADIABATIC = 2 };
enum { WEST = 0, EAST = 1, SOUTH = 2, NORTH = 3 };

typedef struct {
    int nx, ny;
    int kind[4];       /* per edge: periodic / Dirichlet-temperature wall / adiabatic wall */
    double uw[4][2];   /* wall velocity per edge */
    double Tw[4];      /* wall temperature per edge (Dirichlet) */
    double T0;         /* reference temperature of Eq. 3 */
    double s_nu, s_b, s3, s4;   /* D2Q9 rates of S */
    double lam1, lam2;          /* D2Q5 rates of S_T (lambda0 acts on a conserved moment) */
    double g_beta, Fvx, Fvy;    /* Eq. 3 */
    int prescribed;             /* 1: velocity is given (Sec. 3.1); only the D2Q5 equation runs */
    double pux, puy;            /* the given velocity */
    double *f, *g;              /* state(t) */
    double *fn, *gn;            /* next state */
    double *out;                /* f*_k sent out of the domain by wall nodes in the last step */
    double Minv[81], MTinv[25];
    int bad;                    /* set when a NaN survives the wall step */
} orc_lattice;

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
    double a[81 * 2];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < 2 * n; ++j)
            a[i * 2 * n + j] = (j < n) ? A[i * n + j] : (j - n == i ? 1.0 : 0.0);
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(a[r * 2 * n + c]) > fabs(a[p * 2 * n + c])) p = r;
        if (a[p * 2 * n + c] == 0.0) return -1;
        if (p != c)
            for (int j = 0; j < 2 * n; ++j) {
                double t = a[c * 2 * n + j];
                a[c * 2 * n + j] = a[p * 2 * n + j];
                a[p * 2 * n + j] = t;
            }
        double piv = a[c * 2 * n + c];
        for (int j = 0; j < 2 * n; ++j) a[c * 2 * n + j] /= piv;
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            double m = a[r * 2 * n + c];
            if (m != 0.0)
                for (int j = 0; j < 2 * n; ++j) a[r * 2 * n + j] -= m * a[c * 2 * n + j];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Ainv[i * n + j] = a[i * 2 * n + n + j];
    return 0;
}

/* Solve L x = b for a unit lower-triangular L (forward substitution).  N of Eq. 7b and N_T of
 * Eq. 18 are unit lower triangular as printed, so this applies N^-1 and N_T^-1. */
static void solve_unit_lower(int n, const double* L, const double* b, double* x)
{
    for (int i = 0; i < n; ++i) {
        double s = b[i];
        for (int j = 0; j < i; ++j) s -= L[i * n + j] * x[j];
        x[i] = s;
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Sec. 2.1 matrices.                                                                          */

/* Eq. 7a: Gamma = M f, with Gamma = [k00,k10,k01,k20,k02,k11,k21,k12,k22] (Eq. 6). */
static const double M9[81] = {
    1, 1, 1, 1, 1, 1, 1, 1, 1,
    0, 1, 0, -1, 0, 1, -1, -1, 1,
    0, 0, 1, 0, -1, 1, 1, -1, -1,
    0, 1, 0, 1, 0, 1, 1, 1, 1,
    0, 0, 1, 0, 1, 1, 1, 1, 1,
    0, 0, 0, 0, 0, 1, -1, 1, -1,
    0, 0, 0, 0, 0, 1, 1, -1, -1,
    0, 0, 0, 0, 0, 1, -1, -1, 1,
    0, 0, 0, 0, 0, 1, 1, 1, 1,
};

/* Eq. 7b: Gamma~ = N(u) Gamma.  Row k~02 uses -2 u_y (see the header). */
static void build_N(double ux, double uy, double* N)
{
    const double ux2 = ux * ux, uy2 = uy * uy;
    const double rows[81] = {
        1, 0, 0, 0, 0, 0, 0, 0, 0,
        -ux, 1, 0, 0, 0, 0, 0, 0, 0,
        -uy, 0, 1, 0, 0, 0, 0, 0, 0,
        ux2, -2 * ux, 0, 1, 0, 0, 0, 0, 0,
        uy2, 0, -2 * uy, 0, 1, 0, 0, 0, 0,
        ux * uy, -uy, -ux, 0, 0, 1, 0, 0, 0,
        -ux2 * uy, 2 * ux * uy, ux2, -uy, 0, -2 * ux, 1, 0, 0,
        -uy2 * ux, uy2, 2 * ux * uy, 0, -ux, -2 * uy, 0, 1, 0,
        ux2 * uy2, -2 * ux * uy2, -2 * uy * ux2, uy2, ux2, 4 * ux * uy, -2 * uy, -2 * ux, 1,
    };
    memcpy(N, rows, sizeof rows);
}

/* Relaxation matrix S of Eq. 8: diag([0,0,0], [[s+,s-],[s-,s+]], [s_nu,s3,s3,s4]),
 * s+ = (s_b + s_nu)/2, s- = (s_b - s_nu)/2. */
static void build_S(const orc_lattice* L, double* S)
{
    memset(S, 0, 81 * sizeof(double));
    const double sp = 0.5 * (L->s_b + L->s_nu), sm = 0.5 * (L->s_b - L->s_nu);
    S[3 * 9 + 3] = sp; S[3 * 9 + 4] = sm;
    S[4 * 9 + 3] = sm; S[4 * 9 + 4] = sp;
    S[5 * 9 + 5] = L->s_nu;
    S[6 * 9 + 6] = L->s3;
    S[7 * 9 + 7] = L->s3;
    S[8 * 9 + 8] = L->s4;
}

/* ------------------------------------------------------------------------------------------ */
/* Sec. 2.2 matrices.                                                                          */

/* Eq. 17: Gamma_T = M_T g, Gamma_T = [k00,k10,k01,k20,k02] (Eq. 15). */
static const double M5[25] = {
    1, 1, 1, 1, 1,
    0, 1, 0, -1, 0,
    0, 0, 1, 0, -1,
    0, 1, 0, 1, 0,
    0, 0, 1, 0, 1,
};

/* Eq. 18: Gamma~_T = N_T(u) Gamma_T. */
static void build_NT(double ux, double uy, double* N)
{
    const double rows[25] = {
        1, 0, 0, 0, 0,
        -ux, 1, 0, 0, 0,
        -uy, 0, 1, 0, 0,
        ux * ux, -2 * ux, 0, 1, 0,
        uy * uy, 0, -2 * uy, 0, 1,
    };
    memcpy(N, rows, sizeof rows);
}

/* ------------------------------------------------------------------------------------------ */
/* Equilibria.  The equilibrium populations are those whose central moments are Eq. 9 (D2Q9)
 * and Eq. 20 (D2Q5): f^eq = M^-1 N(u)^-1 Gamma~^eq, g^eq = M_T^-1 N_T(u)^-1 Gamma~_T^eq.        */

static void feq9(const orc_lattice* L, double rho, double ux, double uy, double* out)
{
    const double Geq[9] = {rho, 0, 0, rho * CS2, rho * CS2, 0, 0, 0, rho * CS2 * CS2};
    double N[81], G[9];
    build_N(ux, uy, N);
    solve_unit_lower(9, N, Geq, G);
    matvec(9, L->Minv, G, out);
}

static void geq5(const orc_lattice* L, double T, double ux, double uy, double* out)
{
    const double Geq[5] = {T, 0, 0, T * CT2, T * CT2};
    double N[25], G[5];
    build_NT(ux, uy, N);
    solve_unit_lower(5, N, Geq, G);
    matvec(5, L->MTinv, G, out);
}

/* ------------------------------------------------------------------------------------------ */
/* Collisions.                                                                                  */

/* Eq. 8 for one node: Gamma = M f, Gamma~ = N Gamma,
 * Gamma~* = (I - S) Gamma~ + S Gamma~^eq + (I - S/2) C,  f* = M^-1 N^-1 Gamma~*. */
static void collide9(const orc_lattice* L, const double* f, double rho, double ux, double uy,
                     double Fx, double Fy, double* fpost)
{
    double N[81], S[81], G[9], Gt[9], Gs[9], Graw[9];
    const double Geq[9] = {rho, 0, 0, rho * CS2, rho * CS2, 0, 0, 0, rho * CS2 * CS2}; /* Eq. 9 */
    const double C[9] = {0, Fx, Fy, 0, 0, 0, CS2 * Fy, CS2 * Fx, 0};                   /* Eq. 11 */
    matvec(9, M9, f, G);
    build_N(ux, uy, N);
    matvec(9, N, G, Gt);
    build_S(L, S);
    for (int i = 0; i < 9; ++i) {
        double s = 0.0;
        for (int j = 0; j < 9; ++j) {
            const double I = (i == j) ? 1.0 : 0.0;
            s += (I - S[i * 9 + j]) * Gt[j] + S[i * 9 + j] * Geq[j] + (I - 0.5 * S[i * 9 + j]) * C[j];
        }
        Gs[i] = s;
    }
    solve_unit_lower(9, N, Gs, Graw);
    matvec(9, L->Minv, Graw, fpost);
}

/* Eq. 19 for one node: Gamma~_T* = (I - S_T) Gamma~_T + S_T Gamma~_T^eq,
 * g* = M_T^-1 N_T^-1 Gamma~_T* (Eq. 21).  S_T = diag(lambda0, lambda1, lambda1, lambda2, lambda2);
 * lambda0 multiplies k~00 - T = 0, so its value does not matter; 1 is used. */
static void collide5(const orc_lattice* L, const double* g, double T, double ux, double uy, double* gpost)
{
    double N[25], G[5], Gt[5], Gs[5], Graw[5];
    const double Geq[5] = {T, 0, 0, T * CT2, T * CT2}; /* Eq. 20 */
    const double ST[5] = {1.0, L->lam1, L->lam1, L->lam2, L->lam2};
    matvec(5, M5, g, G);
    build_NT(ux, uy, N);
    matvec(5, N, G, Gt);
    for (int i = 0; i < 5; ++i) Gs[i] = (1.0 - ST[i]) * Gt[i] + ST[i] * Geq[i];
    solve_unit_lower(5, N, Gs, Graw);
    matvec(5, L->MTinv, Graw, gpost);
}

/* ------------------------------------------------------------------------------------------ */
/* Macroscopic quantities: Eq. 23 (T), Eq. 3 (F), Eq. 13 (rho, u).                              */

static void force_of(const orc_lattice* L, double T, double* Fx, double* Fy)
{
    *Fx = L->Fvx;
    *Fy = L->Fvy + L->g_beta * (T - L->T0);
}

static void macro_of(const orc_lattice* L, const double* f, const double* g, double* rho,
                     double* ux, double* uy, double* T, double* Fx, double* Fy)
{
    double t = 0.0;
    for (int i = 0; i < 5; ++i) t += g[i];
    *T = t;
    force_of(L, t, Fx, Fy);
    if (L->prescribed) {
        *rho = 1.0;
        *ux = L->pux;
        *uy = L->puy;
        return;
    }
    double r = 0.0, jx = 0.0, jy = 0.0;
    for (int i = 0; i < 9; ++i) {
        r += f[i];
        jx += f[i] * EX[i];
        jy += f[i] * EY[i];
    }
    *rho = r;
    *ux = (jx + 0.5 * (*Fx)) / r;
    *uy = (jy + 0.5 * (*Fy)) / r;
}

/* ------------------------------------------------------------------------------------------ */
/* Wall step.                                                                                   */

static int idx_of(const orc_lattice* L, int x, int y) { return y * L->nx + x; }

static void load_node(const orc_lattice* L, int x, int y, double* f, double* g)
{
    const int n = L->nx * L->ny, k = idx_of(L, x, y);
    for (int i = 0; i < 9; ++i) f[i] = L->f[i * n + k];
    for (int i = 0; i < 5; ++i) g[i] = L->g[i * n + k];
}

/* Index of the lattice direction equal to (ex, ey). */
static int dir_of(int ex, int ey)
{
    for (int i = 0; i < 9; ++i)
        if (EX[i] == ex && EY[i] == ey) return i;
    return -1;
}

/* Force-corrected non-equilibrium bounce-back (Zou-He) on a straight wall, in the wall's own
 * frame: n is the inward unit normal, t the tangent with (t, n) a right-handed pair.  The three
 * populations with e.n = +1 are unknown.  The closure bounces back the non-equilibrium part of the
 * normal population, f(0,+1) - f(0,-1) = f^eq(0,+1) - f^eq(0,-1) at (rho, u_w), and fixes the two
 * diagonal ones so that sum f e = rho u_w - F/2, which makes Eq. 13 return u_w.
 *
 * zou_he_density: Zou-He's own density, the one for which in addition sum f = rho:
 * rho = (sum_{b=0} f + 2 sum_{b=-1} f - F_n/2) / (1 - u_n).
 * zou_he: the three unknowns for a given density rho. */
static double zou_he_density(const double* f, int nx_, int ny_, double uwx, double uwy, double Fx, double Fy)
{
    const int tx = ny_, ty = -nx_;          /* t = n rotated by -90 degrees */
#define D(a, b) dir_of((a) * tx + (b) * nx_, (a) * ty + (b) * ny_)
    const double K0 = f[D(0, 0)] + f[D(1, 0)] + f[D(-1, 0)];
    const double Km = f[D(0, -1)] + f[D(1, -1)] + f[D(-1, -1)];
#undef D
    const double un = uwx * nx_ + uwy * ny_;
    const double Fn = Fx * nx_ + Fy * ny_;
    return (K0 + 2.0 * Km - 0.5 * Fn) / (1.0 - un);
}

static void zou_he(double* f, int nx_, int ny_, double uwx, double uwy, double Fx, double Fy, double rho)
{
    const int tx = ny_, ty = -nx_;          /* t = n rotated by -90 degrees */
#define D(a, b) dir_of((a) * tx + (b) * nx_, (a) * ty + (b) * ny_)
    const int cp0 = D(1, 0), cm0 = D(-1, 0);
    const int c0m = D(0, -1), cpm = D(1, -1), cmm = D(-1, -1);
    const int c0p = D(0, 1), cpp = D(1, 1), cmp = D(-1, 1);
#undef D
    const double un = uwx * nx_ + uwy * ny_, ut = uwx * tx + uwy * ty;
    const double Fn = Fx * nx_ + Fy * ny_, Ft = Fx * tx + Fy * ty;
    const double Dn = rho * un * (2.0 / 3.0 - ut * ut);
    f[c0p] = f[c0m] + Dn;
    f[cpp] = f[cmm] - 0.5 * (f[cp0] - f[cm0]) + 0.5 * (rho * ut - 0.5 * Ft) + 0.5 * (rho * un - 0.5 * Fn - Dn);
    f[cmp] = f[cpm] + 0.5 * (f[cp0] - f[cm0]) - 0.5 * (rho * ut - 0.5 * Ft) + 0.5 * (rho * un - 0.5 * Fn - Dn);
}

/* Wall step at node (x, y): replaces the unknown populations of f (and, on impermeable walls,
 * the rest population f_0) and all of g in place. */
static void wall_step(const orc_lattice* L, int x, int y, double* f, double* g)
{
    const int onW = L->kind[WEST] != W_PERIODIC && x == 0;
    const int onE = L->kind[EAST] != W_PERIODIC && x == L->nx - 1;
    const int onS = L->kind[SOUTH] != W_PERIODIC && y == 0;
    const int onN = L->kind[NORTH] != W_PERIODIC && y == L->ny - 1;
    if (!(onW || onE || onS || onN)) return;
    const int xwall = onW ? WEST : (onE ? EAST : -1);
    const int ywall = onS ? SOUTH : (onN ? NORTH : -1);
    const int corner = xwall >= 0 && ywall >= 0;
    const int dx = onW ? 1 : (onE ? -1 : 0);
    const int dy = onS ? 1 : (onN ? -1 : 0);

    /* Wall data.  Velocity: the west/east wall's at a corner.  Temperature: Dirichlet wins. */
    const int vw = xwall >= 0 ? xwall : ywall;
    int tw;
    if (xwall >= 0 && ywall >= 0)
        tw = (L->kind[xwall] == W_DIRICHLET || L->kind[ywall] != W_DIRICHLET) ? xwall : ywall;
    else
        tw = vw;
    double uwx = L->uw[vw][0], uwy = L->uw[vw][1];
    if (L->prescribed) { uwx = L->pux; uwy = L->puy; }

    /* Inner neighbour x_f (the diagonal one at a corner) and its post-streaming macroscopic state. */
    double ff[9], gf[5], rf, uxf, uyf, Tf, Fxf, Fyf;
    load_node(L, x + dx, y + dy, ff, gf);
    macro_of(L, ff, gf, &rf, &uxf, &uyf, &Tf, &Fxf, &Fyf);

    /* (1a) temperature: non-equilibrium extrapolation, all five g replaced. */
    double Tb;
    if (L->kind[tw] == W_DIRICHLET) {
        Tb = L->Tw[tw];
    } else {
        double fff[9], gff[5], Tff = 0.0;
        load_node(L, x + 2 * dx, y + 2 * dy, fff, gff);
        for (int i = 0; i < 5; ++i) Tff += gff[i];
        Tb = (4.0 * Tf - Tff) / 3.0;
    }
    double gb[5], gfe[5];
    geq5(L, Tb, uwx, uwy, gb);
    geq5(L, Tf, uxf, uyf, gfe);
    for (int i = 0; i < 5; ++i) g[i] = gb[i] + (gf[i] - gfe[i]);
    if (L->prescribed) return;

    /* (1b) force at the wall node from its temperature. */
    double Fxb, Fyb;
    force_of(L, Tb, &Fxb, &Fyb);

    /* (1c) density of the wall node.  Population i is unknown when its source x - e_i lies beyond
     * a wall (after streaming those entries of state(t) are NaN; the initial state holds values
     * there, which the wall step replaces all the same); the populations the node sent out of the
     * domain last step are out[opp(i)] for those i. */
    const int n = L->nx * L->ny, k = idx_of(L, x, y);
    const int impermeable = corner || (uwx * dx + uwy * dy == 0.0);
    int unknown[9];
    double rho_b;
    for (int i = 0; i < 9; ++i)
        unknown[i] = (onW && EX[i] > 0) || (onE && EX[i] < 0) || (onS && EY[i] > 0) || (onN && EY[i] < 0);
    if (impermeable) {
        rho_b = 0.0;
        for (int i = 0; i < 9; ++i) rho_b += unknown[i] ? L->out[OPP[i] * n + k] : f[i];
    } else {
        rho_b = zou_he_density(f, dx, dy, uwx, uwy, Fxb, Fyb);
    }

    if (!corner) {
        /* (1d) Zou-He on the edge; the inward normal is (dx, dy). */
        zou_he(f, dx, dy, uwx, uwy, Fxb, Fyb, rho_b);
    } else {
        /* (1d) corner: five unknowns.  Those whose opposite is known bounce back the opposite's
         * non-equilibrium part, f_i = f_opp(i) + f_i^eq - f_opp(i)^eq; the two whose opposite is
         * unknown too (they point along the diagonal the corner cuts off) take f_i^eq.  The
         * equilibrium is at (rho_b, u_w - F_b/(2 rho_b)), whose first moment is rho_b u_w - F_b/2,
         * so Eq. 13 returns u_w at the corner. */
        double fe[9];
        feq9(L, rho_b, uwx - 0.5 * Fxb / rho_b, uwy - 0.5 * Fyb / rho_b, fe);
        for (int i = 1; i < 9; ++i) {
            if (!unknown[i]) continue;
            f[i] = unknown[OPP[i]] ? fe[i] : f[OPP[i]] + (fe[i] - fe[OPP[i]]);
        }
    }
    if (impermeable) {
        /* (1e) the rest population carries the mass balance: sum f = rho_b. */
        double s = 0.0;
        for (int i = 1; i < 9; ++i) s += f[i];
        f[0] = rho_b - s;
    }
}

/* Wall step + macroscopic step at one node (steps 1-2 of a time step). */
static void pre_collision(orc_lattice* L, int x, int y, double* f, double* g, double* rho,
                          double* ux, double* uy, double* T, double* Fx, double* Fy)
{
    load_node(L, x, y, f, g);
    wall_step(L, x, y, f, g);
    int nan_left = 0;
    for (int i = 0; i < 5; ++i) nan_left |= isnan(g[i]);
    if (!L->prescribed)
        for (int i = 0; i < 9; ++i) nan_left |= isnan(f[i]);
    if (nan_left) {
#pragma omp atomic write
        L->bad = 1;
    }
    macro_of(L, f, g, rho, ux, uy, T, Fx, Fy);
}

/* ------------------------------------------------------------------------------------------ */
/* Public C interface (loaded with ctypes by the tests).                                        */

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for the following steps (n >= 1); used to time the oracle on one core. */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

orc_lattice* orc_create(int nx, int ny, const int* kind, const double* uw, const double* Tw, double T0)
{
    if (nx < 3 || ny < 3) return NULL;
    if ((kind[WEST] == W_PERIODIC) != (kind[EAST] == W_PERIODIC)) return NULL;
    if ((kind[SOUTH] == W_PERIODIC) != (kind[NORTH] == W_PERIODIC)) return NULL;
    orc_lattice* L = (orc_lattice*)calloc(1, sizeof(orc_lattice));
    if (!L) return NULL;
    L->nx = nx;
    L->ny = ny;
    for (int e = 0; e < 4; ++e) {
        L->kind[e] = kind[e];
        L->uw[e][0] = uw[2 * e];
        L->uw[e][1] = uw[2 * e + 1];
        L->Tw[e] = Tw[e];
    }
    L->T0 = T0;
    L->s_nu = 1.0; L->s_b = 1.0; L->s3 = 1.0; L->s4 = 1.0;
    L->lam1 = 1.0; L->lam2 = 1.0;
    const size_t n = (size_t)nx * ny;
    L->f = (double*)malloc(9 * n * sizeof(double));
    L->fn = (double*)malloc(9 * n * sizeof(double));
    L->g = (double*)malloc(5 * n * sizeof(double));
    L->gn = (double*)malloc(5 * n * sizeof(double));
    L->out = (double*)malloc(9 * n * sizeof(double));
    if (!L->f || !L->fn || !L->g || !L->gn || !L->out || invert(9, M9, L->Minv) || invert(5, M5, L->MTinv)) {
        free(L->f); free(L->fn); free(L->g); free(L->gn); free(L->out); free(L);
        return NULL;
    }
    for (size_t i = 0; i < 9 * n; ++i) L->out[i] = NAN;
    for (size_t i = 0; i < 9 * n; ++i) L->f[i] = NAN;
    for (size_t i = 0; i < 5 * n; ++i) L->g[i] = NAN;
    return L;
}

void orc_destroy(orc_lattice* L)
{
    if (!L) return;
    free(L->f); free(L->fn); free(L->g); free(L->gn); free(L->out);
    free(L);
}

/* tau_nu = 1/s_nu (nu = (tau_nu - 1/2)/3, Sec. 2.1); tau_alpha = 1/lambda1
 * (alpha = (tau_alpha - 1/2) c_{T,s}^2, Sec. 2.2). */
void orc_set_params(orc_lattice* L, double tau_nu, double tau_alpha, double g_beta)
{
    L->s_nu = 1.0 / tau_nu;
    L->lam1 = 1.0 / tau_alpha;
    L->g_beta = g_beta;
}

void orc_set_relaxation(orc_lattice* L, double s_b, double s3, double s4, double lam2)
{
    L->s_b = s_b; L->s3 = s3; L->s4 = s4; L->lam2 = lam2;
}

void orc_set_body_force(orc_lattice* L, double Fvx, double Fvy) { L->Fvx = Fvx; L->Fvy = Fvy; }

void orc_set_prescribed_velocity(orc_lattice* L, int on, double ux, double uy)
{
    L->prescribed = on; L->pux = ux; L->puy = uy;
}

/* Initial state: g = g^eq(T, u0), f = f^eq(rho0, u0 - F/(2 rho0)) with F from T (Eq. 3), so that
 * Eq. 13 returns (rho0, u0) and Eq. 23 returns T.  NULL arrays mean rho = 1, u = 0, T = T0.
 * The outgoing populations of the step before t = 0 are taken as the initial values of the
 * unknown populations they pair with, out[opp(i)] = f_i, so that a wall node's mass balance
 * returns rho0. */
void orc_init(orc_lattice* L, const double* rho, const double* ux, const double* uy, const double* T)
{
    const int n = L->nx * L->ny;
    for (int k = 0; k < n; ++k) {
        const double r = rho ? rho[k] : 1.0;
        double u = ux ? ux[k] : 0.0, v = uy ? uy[k] : 0.0;
        const double t = T ? T[k] : L->T0;
        if (L->prescribed) { u = L->pux; v = L->puy; }
        double Fx, Fy, fe[9], ge[5];
        force_of(L, t, &Fx, &Fy);
        feq9(L, r, u - 0.5 * Fx / r, v - 0.5 * Fy / r, fe);
        geq5(L, t, u, v, ge);
        for (int i = 0; i < 9; ++i) L->f[i * n + k] = fe[i];
        for (int i = 0; i < 5; ++i) L->g[i * n + k] = ge[i];
        for (int i = 0; i < 9; ++i) L->out[OPP[i] * n + k] = fe[i];
    }
    L->bad = 0;
}

/* n time steps.  Returns 0, or -1 if a population that should have been reconstructed by the
 * wall step was still unknown (NaN), which would mean the wall step is incomplete. */
int orc_step(orc_lattice* L, long long nsteps)
{
    const int nx = L->nx, ny = L->ny, n = nx * ny;
    for (long long s = 0; s < nsteps; ++s) {
        for (int i = 0; i < 9 * n; ++i) L->fn[i] = NAN;
        for (int i = 0; i < 5 * n; ++i) L->gn[i] = NAN;
#pragma omp parallel for schedule(static)
        for (int y = 0; y < ny; ++y) {
            for (int x = 0; x < nx; ++x) {
                double f[9], g[5], fp[9], gp[5], rho, ux, uy, T, Fx, Fy;
                pre_collision(L, x, y, f, g, &rho, &ux, &uy, &T, &Fx, &Fy);
                if (!L->prescribed) collide9(L, f, rho, ux, uy, Fx, Fy, fp);
                collide5(L, g, T, ux, uy, gp);
                /* Eqs. 12 and 22: f_i(x + e_i, t + 1) = f_i*(x, t); targets outside a wall are dropped. */
                for (int i = 0; i < 9; ++i) {
                    int tx = x + EX[i], ty = y + EY[i];
                    if (L->kind[WEST] == W_PERIODIC) tx = (tx + nx) % nx;
                    if (L->kind[SOUTH] == W_PERIODIC) ty = (ty + ny) % ny;
                    if (tx < 0 || tx >= nx || ty < 0 || ty >= ny) {
                        if (!L->prescribed) L->out[i * n + y * nx + x] = fp[i];
                        continue;
                    }
                    const int t = ty * nx + tx;
                    if (!L->prescribed) L->fn[i * n + t] = fp[i];
                    if (i < 5) L->gn[i * n + t] = gp[i];
                }
            }
        }
        double* tmp = L->f; L->f = L->fn; L->fn = tmp;
        tmp = L->g; L->g = L->gn; L->gn = tmp;
    }
    return L->bad ? -1 : 0;
}

/* rho, u, T of the current time: the wall step and Eqs. 3, 13, 23 applied to state(t). */
int orc_moments(orc_lattice* L, double* rho, double* ux, double* uy, double* T)
{
    const int nx = L->nx, ny = L->ny;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            double f[9], g[5], r, u, v, t, Fx, Fy;
            pre_collision(L, x, y, f, g, &r, &u, &v, &t, &Fx, &Fy);
            const int k = y * nx + x;
            if (rho) rho[k] = r;
            if (ux) ux[k] = u;
            if (uy) uy[k] = v;
            if (T) T[k] = t;
        }
    return L->bad ? -1 : 0;
}

/* Copy out / in state(t): f as [9][ny][nx], g as [5][ny][nx]; unknown entries are NaN. */
void orc_get_state(const orc_lattice* L, double* f, double* g)
{
    const size_t n = (size_t)L->nx * L->ny;
    if (f) memcpy(f, L->f, 9 * n * sizeof(double));
    if (g) memcpy(g, L->g, 5 * n * sizeof(double));
}

void orc_set_state(orc_lattice* L, const double* f, const double* g)
{
    const size_t n = (size_t)L->nx * L->ny;
    if (f) memcpy(L->f, f, 9 * n * sizeof(double));
    if (g) memcpy(L->g, g, 5 * n * sizeof(double));
    L->bad = 0;
}

/* Copy out / in the outgoing populations out[9][ny][nx] (see the state convention). */
void orc_get_outgoing(const orc_lattice* L, double* out)
{
    memcpy(out, L->out, 9 * (size_t)L->nx * L->ny * sizeof(double));
}

void orc_set_outgoing(orc_lattice* L, const double* out)
{
    memcpy(L->out, out, 9 * (size_t)L->nx * L->ny * sizeof(double));
}

/* ---- single-node access for the algebra tests ---- */
void orc_matrix_M(double* out) { memcpy(out, M9, sizeof M9); }
void orc_matrix_N(double ux, double uy, double* out) { build_N(ux, uy, out); }
void orc_matrix_Minv(const orc_lattice* L, double* out) { memcpy(out, L->Minv, sizeof L->Minv); }
void orc_matrix_S(const orc_lattice* L, double* out) { build_S(L, out); }
void orc_matrix_MT(double* out) { memcpy(out, M5, sizeof M5); }
void orc_matrix_NT(double ux, double uy, double* out) { build_NT(ux, uy, out); }
void orc_matrix_MTinv(const orc_lattice* L, double* out) { memcpy(out, L->MTinv, sizeof L->MTinv); }

/* N_T(u)^-1 column by column through the same forward substitution the collision uses. */
void orc_matrix_NTinv(double ux, double uy, double* out)
{
    double N[25];
    build_NT(ux, uy, N);
    for (int j = 0; j < 5; ++j) {
        double e[5] = {0, 0, 0, 0, 0}, c[5];
        e[j] = 1.0;
        solve_unit_lower(5, N, e, c);
        for (int i = 0; i < 5; ++i) out[i * 5 + j] = c[i];
    }
}

void orc_matrix_Ninv(double ux, double uy, double* out)
{
    double N[81];
    build_N(ux, uy, N);
    for (int j = 0; j < 9; ++j) {
        double e[9] = {0}, c[9];
        e[j] = 1.0;
        solve_unit_lower(9, N, e, c);
        for (int i = 0; i < 9; ++i) out[i * 9 + j] = c[i];
    }
}

void orc_feq(const orc_lattice* L, double rho, double ux, double uy, double* out) { feq9(L, rho, ux, uy, out); }
void orc_geq(const orc_lattice* L, double T, double ux, double uy, double* out) { geq5(L, T, ux, uy, out); }

/* Collision of one node given its pre-collision f and the force: rho, u from Eq. 13. */
void orc_collide9(const orc_lattice* L, const double* f, double Fx, double Fy, double* out)
{
    double r = 0.0, jx = 0.0, jy = 0.0;
    for (int i = 0; i < 9; ++i) { r += f[i]; jx += f[i] * EX[i]; jy += f[i] * EY[i]; }
    collide9(L, f, r, (jx + 0.5 * Fx) / r, (jy + 0.5 * Fy) / r, Fx, Fy, out);
}

void orc_collide5(const orc_lattice* L, const double* g, double ux, double uy, double* out)
{
    double T = 0.0;
    for (int i = 0; i < 5; ++i) T += g[i];
    collide5(L, g, T, ux, uy, out);
}

/* Zou-He closure alone, for the closure tests: inward normal (nx_, ny_), Zou-He's own density. */
void orc_zou_he(double* f, int nx_, int ny_, double uwx, double uwy, double Fx, double Fy)
{
    zou_he(f, nx_, ny_, uwx, uwy, Fx, Fy, zou_he_density(f, nx_, ny_, uwx, uwy, Fx, Fy));
}
