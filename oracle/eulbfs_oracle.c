/*
 * FP64 CPU oracle of the EULBFS time step (enthalpy-based unified lattice
 * Boltzmann flux solver for liquid solidification, arXiv 2507.03366).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file: only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header, table or helper with the HIP
 * library.  It is deliberately slow and literal: every face loops over the
 * lattice directions alpha one by one, builds each equilibrium from its
 * defining equation, forms the non-equilibrium parts and the "star"
 * distributions, and only then takes the moments of Eq. (53).  Nothing is
 * collapsed algebraically, fused or reordered.
 *
 * Paper sections followed (equation numbers are the paper's):
 *   closure H -> (F_l, T)            Sec. 2.1.1, Eqs. (5)-(6)
 *   mixture rule                     Sec. 2.1.1, Eq. (7)
 *   h^eq, D2Q9 velocities            Sec. 2.1.2, Eqs. (9)-(10)
 *   tau_h, C_p,ref                   Sec. 2.1.2 (text after Eq. 8), App. A Eq. (A-11)
 *   f^eq, tau_f                      Sec. 2.2.3, Eq. (29)
 *   f^eq-m                           Sec. 2.2.3, Eqs. (33)-(35)
 *   f*, h*, g*                       Eqs. (13), (16), (35), (37), (44), (46)
 *   mu_c, beta, kappa                Sec. 2.3.1 (text after Eq. 40)
 *   g^eq, tau_g                      Sec. 2.3.2, Eqs. (41)-(42)
 *   W, F, F_E                        Sec. 2.4, Eqs. (48)-(53)
 *   local reconstruction             Sec. 2.4, Eq. (54)
 *   face state at the new level      Sec. 2.4, Eqs. (55)-(56)
 *   SSP-RK3                          Sec. 2.4, Eqs. (57)-(58)
 *   procedure                        Sec. 2.5, steps (1)-(7)
 *
 * Readings where the paper is silent, garbled or self-contradictory (each is
 * a choice shared with the GPU library by specification, not by code):
 *   R1  D2Q9 weights 4/9, 1/9, 1/36 and c_s^2 = 1/3 (never printed); the
 *       optional D2Q5 lattice for h and g uses 1/3, 1/6 and c_s^2 = 1/3.
 *   R2  f* = f^eq(x_f) + (1 - 1/(2 tau_f)) f^neq-m (Eq. 37 prints "-", which
 *       makes the momentum flux anti-viscous; "+" is the sign of Eqs. 16, 46).
 *   R3  mu_c = 2 beta C (C-1)(2C-1) - kappa lap(C) (the printed "+" does not
 *       make the tanh profile of Eq. 61 an equilibrium).
 *   R4  Gamma_alpha of Eq. (34) without the leading "1": f^eq-m is f^eq with
 *       the density taken at the face at the old level (Eq. 33).
 *   R5  The C source of Eqs. (40), (47) is kept as the fifth row of F_E (Eq. 51
 *       prints 0 there).  In Eq. (40) the paper's F_s is 1 - F_l, the solid
 *       share of the condensed phase, and C d(1 - F_l)/dt is the rate at which
 *       the cell's volume turns solid, d(C (1 - F_l))/dt where the condensed
 *       fraction of a freezing cell is steady.  The source is therefore taken
 *       as (1 - rho_s/rho_l) dF_s/dt with the cell's solid fraction F_s =
 *       C (1 - F_l) of R7, the same lagged rate that drives the volume source
 *       of Eqs. (25)-(26): the condensed volume then grows by exactly the
 *       dilatation of the freezing material.  c_source = 1 selects the other
 *       reading, C (1 - rho_s/rho_l) dF_s/dt with the cell's F_s; it weights a
 *       freezing cell of the diffuse interface by C^2 and loses (1 - r) times
 *       the integral of C (1 - C) across the interface (xi/4 for the profile of
 *       Eq. 61) from the final condensed volume, which the full-freezing height
 *       of Sec. 3.2 and the volume ratios of Table 5 do not show.
 *   R6  C_p,ref = (C_p,s + C_p,l)/2 as written in the formula (the text calls it
 *       a harmonic mean).
 *   R7  Gas phase: the solid fraction entering Eq. (7) is F_s = C (1 - F_l),
 *       so gas never turns solid.  The enthalpy keeps the paper's form
 *       H = C_p T + L F_l in every phase (the enthalpy flux of Eq. 17 carries
 *       sensible heat only, so a latent term proportional to C would make
 *       liquid advected into a gas cell appear frozen).  H_s = C_p^S T_s,
 *       H_l = C_p^L T_l + L, with C_p^S, C_p^L the Eq. (7) mixtures with
 *       F_s = C and F_s = 0.  For C = 1 this is Eqs. (5)-(7) unchanged.  C is
 *       clamped to [0,1] wherever it enters the closure or a material
 *       property (F_s too).
 *   R8  Gradients: the derivative at the cell centre of the parabola through
 *       the cell and its two neighbours along each direction (second-order
 *       central differences on a uniform mesh); lap(C): the sum over both
 *       directions of that parabola's second derivative (the 5-point stencil
 *       on a uniform mesh).
 *   R9  Points x_f - e_alpha delta_t with e_alpha . n = 0 lie on the face; they
 *       take the average of the two sides' extrapolations.
 *   R10 Reconstructed variables: T, C, F_s, u, v, p, mu_c.  rho and C_p at a
 *       point come from Eq. (7) at that point.  The face values at the old
 *       level (rho, mu, lambda, C_p, T, mu_c) are the averages of the two
 *       sides' extrapolations to the face centre (text after Eq. 54).
 *       (C_p T) at the face at the new level is C_p,face * T_face (old level).
 *   R11 dF_s/dt in the sources is lagged: (F_s^n - F_s^{n-1}) / Delta t, held
 *       through the three RK stages; 0 at the first step.
 *   R12 Rigid solid: after each RK stage the momentum is projected,
 *       M <- (1 - F_s) M (the paper assumes zero solid velocity, Eq. 25).
 *   R13 Boundaries: 3 ghost layers.  Ghost k (k = 1, 2, 3 outward) mirrors the
 *       interior cell k-1 from the wall.  Periodic: copy.  Walls: p even;
 *       no-slip: both momenta odd; free slip: normal odd, tangential even;
 *       outlet: both even.  Adiabatic: H even.  Dirichlet T_w: T_g = 2 T_w -
 *       T_mirror, H_g from the inverse closure.  Wetting (contact angle theta,
 *       90 deg = plain no-flux): C_g = C_mirror + d_k (4/xi) cos(theta)
 *       C_w (1 - C_w), C_w the first interior cell, d_k the distance between
 *       the ghost and mirror centres ((2k-1) dx on a uniform mesh).  Corners:
 *       x rule on the interior rows first, then the y rule on every column.
 *       Fluxes on wall faces: F_p = 0 unless the wall is an outlet, F_C = 0
 *       (no flux), F_H = 0 when adiabatic.
 *   R14 Initial state from (T, F_l, C, u, v, p): H = (1-F_l)(H_s + C_p^S (T -
 *       T_s)) + F_l (H_l + C_p^L (T - T_l)), M = rho c_s^2 (u, v) with rho from
 *       the closure of that H.
 *   R23 Contact-angle hysteresis (Sec. 3.5 gives advancing and receding angles
 *       but no rule): a wall with a window [theta_rec, theta_adv] reads the
 *       apparent angle of the first three interior cells along the normal,
 *       cos(theta_app) = -(dC/dn at the wall) / ((4/xi) C_w (1 - C_w)), dC/dn
 *       from the parabola through the three cell centres, and uses theta_app
 *       clamped to the window in place of theta in the wetting rule of R13 (a
 *       contact line inside the window keeps its angle, one outside is driven
 *       to the nearer bound).  Where C_w (1 - C_w) <= 1e-3 (no interface at
 *       the wall) theta is used.
 *   R24 Stretched meshes (Eq. 52 is written for any mesh; the paper runs
 *       uniform ones): a tensor product of column widths w_i and row heights
 *       h_j.  V = w_i h_j, S = h_j on x faces and w_i on y faces; the face
 *       centre lies w/2 from each neighbouring cell centre, so Eq. (54)
 *       extrapolates by w_a/2 and w_b/2 on the two sides; one streaming step
 *       delta_t for the whole mesh, at most half the smallest width.  Ghost
 *       cells take the width of the cell they copy (mirror or periodic
 *       image), so a wall lies midway between a ghost and its mirror and the
 *       wetting offset of R13 uses the distance 2 s between them (s: wall to
 *       mirror centre).  Uniform spacing dx is the case w_i = h_j = dx.
 */
#include "eulbfs_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------------------
 * Lattices.  Eq. (10): e_0 = 0, e_1..4 = (+-1,0),(0,+-1), e_5..8 = (+-1,+-1).
 * ------------------------------------------------------------------------- */
static const double CS2 = 1.0 / 3.0;
static const int Q9_EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int Q9_EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double Q9_W[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                               1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const double Q5_W[5] = {1.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0};

/* indices of the reconstructed variables */
enum { V_T = 0, V_C, V_FS, V_U, V_V, V_P, V_MUC, NV };

typedef struct {
    double W[5];         /* H, p, Mx = rho cs2 u, My = rho cs2 v, C (Eq. 49) */
    double Fl, Fs, rho, mu, lam, cp;
    double val[NV];      /* T, C, F_s, u, v, p, mu_c */
    double grad[NV][2];  /* central differences (R8) */
} cell_t;

static double clamp01(double x) { return x < 0.0 ? 0.0 : (x > 1.0 ? 1.0 : x); }

/* Eq. (7): gamma = F_s g_s + (1-F_s) C g_l + (1-F_s)(1-C) g_g */
static double mix(const double g[3], double C, double Fs)
{
    return Fs * g[0] + (1.0 - Fs) * C * g[1] + (1.0 - Fs) * (1.0 - C) * g[2];
}

/* Eqs. (5)-(6) with reading R7. */
void or_closure(const or_params* P, double H, double C, double* Fl, double* T)
{
    double Cc = clamp01(C);
    double cpS = mix(P->cp, Cc, Cc);  /* fully solid condensed phase */
    double cpL = mix(P->cp, Cc, 0.0); /* fully liquid condensed phase */
    double Hs = cpS * P->T_s;
    double Hl = cpL * P->T_l + P->latent;
    if (H < Hs) {
        *Fl = 0.0;
        *T = P->T_s + (H - Hs) / cpS;
    } else if (H > Hl) {
        *Fl = 1.0;
        *T = P->T_l + (H - Hl) / cpL;
    } else {
        double f = (Hl - Hs > 1e-300) ? (H - Hs) / (Hl - Hs) : 1.0;
        *Fl = f;
        *T = P->T_s + f * (P->T_l - P->T_s);
    }
}

/* Enthalpy of a state with temperature T and liquid fraction Fl (R14). */
static double enthalpy_of(const or_params* P, double T, double Fl, double C)
{
    double Cc = clamp01(C);
    double cpS = mix(P->cp, Cc, Cc);
    double cpL = mix(P->cp, Cc, 0.0);
    double Hs = cpS * P->T_s;
    double Hl = cpL * P->T_l + P->latent;
    return (1.0 - Fl) * (Hs + cpS * (T - P->T_s)) + Fl * (Hl + cpL * (T - P->T_l));
}

/* Inverse closure used by the Dirichlet ghost cells (R13). */
static double ghost_enthalpy(const or_params* P, double T, double C)
{
    double Fl;
    if (T > P->T_l)
        Fl = 1.0;
    else if (T < P->T_s)
        Fl = 0.0;
    else if (P->T_l > P->T_s)
        Fl = (T - P->T_s) / (P->T_l - P->T_s);
    else
        Fl = 1.0;
    return enthalpy_of(P, T, Fl, C);
}

/* closure + Eq. (7) + velocity for one cell from its conserved vector */
static void derive(const or_params* P, cell_t* c)
{
    double T, Fl;
    or_closure(P, c->W[0], c->W[4], &Fl, &T);
    double Cc = clamp01(c->W[4]);
    c->Fl = Fl;
    c->Fs = Cc * (1.0 - Fl);
    c->rho = mix(P->rho, Cc, c->Fs);
    c->mu = mix(P->mu, Cc, c->Fs);
    c->lam = mix(P->lam, Cc, c->Fs);
    c->cp = mix(P->cp, Cc, c->Fs);
    c->val[V_T] = T;
    c->val[V_C] = c->W[4];
    c->val[V_FS] = c->Fs;
    c->val[V_U] = c->W[2] / (c->rho * CS2);
    c->val[V_V] = c->W[3] / (c->rho * CS2);
    c->val[V_P] = c->W[1];
}

/* ---------------------------------------------------------------------------
 * Equilibria.
 * ------------------------------------------------------------------------- */
/* Eq. (9), alpha >= 1 (alpha = 0 has e = 0 and enters no flux moment). */
static double heq(double w, int ex, int ey, double T, double cp, double cpref, double u, double v)
{
    double eu = ex * u + ey * v;
    double uu = u * u + v * v;
    return w * cp * T * (cpref / cp + eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
}

/* Eq. (29) */
static double feq(double w, int ex, int ey, double p, double rho, double u, double v)
{
    double eu = ex * u + ey * v;
    double uu = u * u + v * v;
    return w * (p + rho * CS2 * (eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2)));
}

/* Eq. (33) with Gamma_alpha of Eq. (34) read as in R4: rho from the face. */
static double feqm(double w, int ex, int ey, double p, double rho_face, double u, double v)
{
    double eu = ex * u + ey * v;
    double uu = u * u + v * v;
    double Gamma = CS2 * (eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
    return w * (p + rho_face * Gamma);
}

/* Eq. (42) */
static double geq(int alpha, double w, int ex, int ey, double C, double muc, double Qg, double u,
                  double v)
{
    if (alpha == 0) return C - muc * Qg * (1.0 - w) / CS2;
    double eu = ex * u + ey * v;
    return w * (muc * Qg + C * eu) / CS2;
}

/* Exposed for the moment tests (Eq. 11 and the analogous moments of f and g). */
void or_equilibria(const or_params* P, double H, double T, double cp, double p, double rho,
                   double C, double muc, double u, double v, double* h_out, double* f_out,
                   double* g_out)
{
    int Qhg = P->lattice_hg == 5 ? 5 : 9;
    const double* Whg = Qhg == 5 ? Q5_W : Q9_W;
    double cpref = 0.5 * (P->cp[0] + P->cp[1]);
    for (int a = 0; a < 9; ++a) f_out[a] = feq(Q9_W[a], Q9_EX[a], Q9_EY[a], p, rho, u, v);
    for (int a = 0; a < Qhg; ++a) {
        if (a == 0) {
            double uu = u * u + v * v;
            h_out[0] = H - cpref * T + Whg[0] * cp * T * (cpref / cp - uu / (2.0 * CS2));
        } else {
            h_out[a] = heq(Whg[a], Q9_EX[a], Q9_EY[a], T, cp, cpref, u, v);
        }
        g_out[a] = geq(a, Whg[a], Q9_EX[a], Q9_EY[a], C, muc, P->Qg, u, v);
    }
}

/* ---------------------------------------------------------------------------
 * Grid with three ghost layers.
 * ------------------------------------------------------------------------- */
#define NG 3

typedef struct {
    const or_params* P;
    int nx, ny, sx; /* sx = nx + 2 NG (row stride) */
    cell_t* c;
    double* wx; /* widths of the nx + 2 NG columns, ghosts included (R24) */
    double* wy; /* heights of the ny + 2 NG rows */
} grid_t;

static cell_t* at(grid_t* g, int i, int j) { return &g->c[(size_t)(j + NG) * g->sx + (i + NG)]; }

static int wrap(int i, int n) { return ((i % n) + n) % n; }

/* width of column i (or height of row i), -NG <= i < n + NG */
static double WX(const grid_t* g, int i) { return g->wx[i + NG]; }
static double WY(const grid_t* g, int j) { return g->wy[j + NG]; }

/* Interior widths from the user array (or dx), ghosts from the cell they copy:
 * the periodic image, or the mirrored interior cell k-1 of ghost layer k (R24). */
static void ghosted_widths(const double* w, double dx, int n, int periodic, double* out)
{
    for (int i = -NG; i < n + NG; ++i) {
        int src;
        if (i >= 0 && i < n)
            src = i;
        else if (periodic)
            src = wrap(i, n);
        else
            src = i < 0 ? -i - 1 : 2 * n - 1 - i;
        out[i + NG] = w ? w[src] : dx;
    }
}

static int grid_alloc(grid_t* g, const or_params* P)
{
    g->P = P;
    g->nx = P->nx;
    g->ny = P->ny;
    g->sx = P->nx + 2 * NG;
    g->c = (cell_t*)calloc((size_t)g->sx * (P->ny + 2 * NG), sizeof(cell_t));
    g->wx = (double*)malloc((size_t)(P->nx + 2 * NG) * sizeof(double));
    g->wy = (double*)malloc((size_t)(P->ny + 2 * NG) * sizeof(double));
    if (!g->c || !g->wx || !g->wy) {
        free(g->c); free(g->wx); free(g->wy);
        return -1;
    }
    ghosted_widths(P->xw, P->dx, P->nx, P->bc[0].periodic, g->wx);
    ghosted_widths(P->yw, P->dx, P->ny, P->bc[2].periodic, g->wy);
    return 0;
}

static void grid_free(grid_t* g)
{
    free(g->c);
    free(g->wx);
    free(g->wy);
}

/* Distances from the wall of `side` to the centres of the first three
 * interior cells along the inward normal. */
static void wall_distances(const grid_t* g, int side, double s[3])
{
    double acc = 0.0;
    for (int m = 0; m < 3; ++m) {
        double w = side == 0 ? WX(g, m) : side == 1 ? WX(g, g->nx - 1 - m) : side == 2 ? WY(g, m) : WY(g, g->ny - 1 - m);
        s[m] = acc + 0.5 * w;
        acc += w;
    }
}

static void load_interior(grid_t* g, const double* W)
{
    size_t n = (size_t)g->nx * g->ny;
    for (int j = 0; j < g->ny; ++j)
        for (int i = 0; i < g->nx; ++i)
            for (int k = 0; k < 5; ++k) at(g, i, j)->W[k] = W[k * n + (size_t)j * g->nx + i];
}

/* Wall rule of R13 applied to one ghost cell.  side: 0 x-, 1 x+, 2 y-, 3 y+.
 * m: the mirrored cell, w, w2, w3: the first three interior cells along the
 * wall normal, whose centres lie s[0], s[1], s[2] from the wall; layer k = 1..3. */
static void wall_ghost(const or_params* P, int side, const cell_t* m, const cell_t* w, const cell_t* w2,
                       const cell_t* w3, const double s[3], int k, double Wg[5])
{
    const or_bc* b = &P->bc[side];
    int normal = side < 2 ? 2 : 3;  /* index of the normal momentum */
    int tang = side < 2 ? 3 : 2;
    Wg[1] = m->W[1];
    if (b->flow == OR_FLOW_NOSLIP) {
        Wg[normal] = -m->W[normal];
        Wg[tang] = -m->W[tang];
    } else if (b->flow == OR_FLOW_FREESLIP) {
        Wg[normal] = -m->W[normal];
        Wg[tang] = m->W[tang];
    } else { /* outlet: zero gradient */
        Wg[normal] = m->W[normal];
        Wg[tang] = m->W[tang];
    }
    /* wetting: dC/dn_in = -(4/xi) cos(theta) C (1 - C) */
    double Cw = w->W[4];
    double d = 2.0 * s[k - 1]; /* ghost centre to mirror centre (R24) */
    double cth = cos(b->theta_deg * M_PI / 180.0);
    if (b->theta_adv > 0.0 && Cw * (1.0 - Cw) > 1e-3) { /* R23 */
        /* dC/dn_in at the wall: derivative at 0 of the Lagrange parabola
         * through (s[0], C_w), (s[1], C_2), (s[2], C_3) */
        double l0 = -(s[1] + s[2]) / ((s[0] - s[1]) * (s[0] - s[2]));
        double l1 = -(s[0] + s[2]) / ((s[1] - s[0]) * (s[1] - s[2]));
        double l2 = -(s[0] + s[1]) / ((s[2] - s[0]) * (s[2] - s[1]));
        double dn = l0 * Cw + l1 * w2->W[4] + l2 * w3->W[4];
        double c_app = -dn / ((4.0 / P->xi) * Cw * (1.0 - Cw));
        double c_adv = cos(b->theta_adv * M_PI / 180.0), c_rec = cos(b->theta_rec * M_PI / 180.0);
        cth = c_app < c_adv ? c_adv : (c_app > c_rec ? c_rec : c_app);
    }
    Wg[4] = m->W[4] + d * (4.0 / P->xi) * cth * Cw * (1.0 - Cw);
    if (b->heat == OR_HEAT_DIRICHLET) {
        double Fl, Tm;
        or_closure(P, m->W[0], m->W[4], &Fl, &Tm);
        double Tg = 2.0 * b->T_w - Tm;
        Wg[0] = ghost_enthalpy(P, Tg, Wg[4]);
    } else {
        Wg[0] = m->W[0];
    }
}

static void fill_ghosts(grid_t* g)
{
    const or_params* P = g->P;
    int nx = g->nx, ny = g->ny;
    double s[4][3];
    for (int side = 0; side < 4; ++side) wall_distances(g, side, s[side]);
    /* x rule on the interior rows */
    for (int j = 0; j < ny; ++j) {
        for (int k = 1; k <= NG; ++k) {
            cell_t* gl = at(g, -k, j);
            cell_t* gr = at(g, nx - 1 + k, j);
            if (P->bc[0].periodic) {
                memcpy(gl->W, at(g, wrap(-k, nx), j)->W, sizeof gl->W);
                memcpy(gr->W, at(g, wrap(nx - 1 + k, nx), j)->W, sizeof gr->W);
            } else {
                wall_ghost(P, 0, at(g, k - 1, j), at(g, 0, j), at(g, 1, j), at(g, 2, j), s[0], k, gl->W);
                wall_ghost(P, 1, at(g, nx - k, j), at(g, nx - 1, j), at(g, nx - 2, j), at(g, nx - 3, j), s[1], k,
                           gr->W);
            }
        }
    }
    /* y rule on every column, ghosts included */
    for (int i = -NG; i < nx + NG; ++i) {
        for (int k = 1; k <= NG; ++k) {
            cell_t* gb = at(g, i, -k);
            cell_t* gt = at(g, i, ny - 1 + k);
            if (P->bc[2].periodic) {
                memcpy(gb->W, at(g, i, wrap(-k, ny))->W, sizeof gb->W);
                memcpy(gt->W, at(g, i, wrap(ny - 1 + k, ny))->W, sizeof gt->W);
            } else {
                wall_ghost(P, 2, at(g, i, k - 1), at(g, i, 0), at(g, i, 1), at(g, i, 2), s[2], k, gb->W);
                wall_ghost(P, 3, at(g, i, ny - k), at(g, i, ny - 1), at(g, i, ny - 2), at(g, i, ny - 3), s[3], k,
                           gt->W);
            }
        }
    }
}

/* R8: first and second derivative at the middle point of the parabola through
 * (-hm, vm), (0, v0), (hp, vp); on a uniform mesh (hm = hp = dx) these are
 * (vp - vm) / (2 dx) and (vp - 2 v0 + vm) / dx^2. */
static double d1(double hm, double hp, double vm, double v0, double vp)
{
    return (hm * hm * (vp - v0) + hp * hp * (v0 - vm)) / (hm * hp * (hm + hp));
}

static double d2(double hm, double hp, double vm, double v0, double vp)
{
    return 2.0 * ((vp - v0) / hp - (v0 - vm) / hm) / (hm + hp);
}

/* centre-to-centre distances to the previous and next column (row) */
static double HXM(const grid_t* g, int i) { return 0.5 * (WX(g, i - 1) + WX(g, i)); }
static double HXP(const grid_t* g, int i) { return 0.5 * (WX(g, i) + WX(g, i + 1)); }
static double HYM(const grid_t* g, int j) { return 0.5 * (WY(g, j - 1) + WY(g, j)); }
static double HYP(const grid_t* g, int j) { return 0.5 * (WY(g, j) + WY(g, j + 1)); }

/* Closure, properties, mu_c and gradients on the whole ghosted grid (steps
 * (2) and (6) of Sec. 2.5 need them at every stage). */
static void derive_all(grid_t* g)
{
    const or_params* P = g->P;
    int nx = g->nx, ny = g->ny;
    double beta = 12.0 * P->sigma / P->xi;
    double kappa = 1.5 * P->xi * P->sigma;
#pragma omp parallel for schedule(static)
    for (int j = -NG; j < ny + NG; ++j)
        for (int i = -NG; i < nx + NG; ++i) derive(P, at(g, i, j));
    /* chemical potential (R3, R8) on interior + 2 ghost layers */
#pragma omp parallel for schedule(static)
    for (int j = -2; j < ny + 2; ++j)
        for (int i = -2; i < nx + 2; ++i) {
            double C = at(g, i, j)->W[4];
            double lap = d2(HXM(g, i), HXP(g, i), at(g, i - 1, j)->W[4], C, at(g, i + 1, j)->W[4]) +
                         d2(HYM(g, j), HYP(g, j), at(g, i, j - 1)->W[4], C, at(g, i, j + 1)->W[4]);
            at(g, i, j)->val[V_MUC] = 2.0 * beta * C * (C - 1.0) * (2.0 * C - 1.0) - kappa * lap;
        }
    /* gradients (R8) on interior + 1 ghost layer */
#pragma omp parallel for schedule(static)
    for (int j = -1; j < ny + 1; ++j)
        for (int i = -1; i < nx + 1; ++i)
            for (int v = 0; v < NV; ++v) {
                at(g, i, j)->grad[v][0] = d1(HXM(g, i), HXP(g, i), at(g, i - 1, j)->val[v], at(g, i, j)->val[v],
                                             at(g, i + 1, j)->val[v]);
                at(g, i, j)->grad[v][1] = d1(HYM(g, j), HYP(g, j), at(g, i, j - 1)->val[v], at(g, i, j)->val[v],
                                             at(g, i, j + 1)->val[v]);
            }
}

/* Eq. (54): psi at the position r (relative to the centre of cell c). */
static void reconstruct(const cell_t* c, double rx, double ry, double out[NV])
{
    for (int v = 0; v < NV; ++v) out[v] = c->val[v] + rx * c->grad[v][0] + ry * c->grad[v][1];
}

/* Fluxes of Eq. (53) through the face between cell a (left or below) and
 * cell b (right or above).  dir 0: x-face (n = +x); dir 1: y-face (n = +y).
 * The face centre lies half_a from the centre of a and half_b from that of b
 * (half the cells' widths along n, R24). */
static void face_flux(const or_params* P, const cell_t* a, const cell_t* b, int dir, double half_a, double half_b,
                      double F[5])
{
    const int Qhg = P->lattice_hg == 5 ? 5 : 9;
    const double* Whg = Qhg == 5 ? Q5_W : Q9_W;
    const double cpref = 0.5 * (P->cp[0] + P->cp[1]); /* R6 */
    const double dt = P->delta_t;
    const int nxn = dir == 0 ? 1 : 0, nyn = dir == 0 ? 0 : 1;

    /* old-level face state: average of both extrapolations to the face centre */
    double ra[NV], rb[NV], avg[NV];
    reconstruct(a, half_a * nxn, half_a * nyn, ra);
    reconstruct(b, -half_b * nxn, -half_b * nyn, rb);
    for (int v = 0; v < NV; ++v) avg[v] = 0.5 * (ra[v] + rb[v]);
    double Cf = clamp01(avg[V_C]), Fsf = clamp01(avg[V_FS]);
    double rho_f = mix(P->rho, Cf, Fsf);
    double mu_f = mix(P->mu, Cf, Fsf);
    double lam_f = mix(P->lam, Cf, Fsf);
    double cp_f = mix(P->cp, Cf, Fsf);
    double T_f = avg[V_T];
    double muc_f = avg[V_MUC];

    /* step (2): the surrounding points x_f - e_alpha delta_t and their equilibria */
    double feq_pt[9], feqm_pt[9], heq_pt[9], geq_pt[9];
    for (int al = 0; al < 9; ++al) {
        int ex = Q9_EX[al], ey = Q9_EY[al];
        int side = ex * nxn + ey * nyn; /* e_alpha . n */
        double psi[NV];
        if (side > 0) {
            reconstruct(a, half_a * nxn - ex * dt, half_a * nyn - ey * dt, psi);
        } else if (side < 0) {
            reconstruct(b, -half_b * nxn - ex * dt, -half_b * nyn - ey * dt, psi);
        } else {
            double pa[NV], pb[NV];
            reconstruct(a, half_a * nxn - ex * dt, half_a * nyn - ey * dt, pa);
            reconstruct(b, -half_b * nxn - ex * dt, -half_b * nyn - ey * dt, pb);
            for (int v = 0; v < NV; ++v) psi[v] = 0.5 * (pa[v] + pb[v]);
        }
        double Cc = clamp01(psi[V_C]), Fs = clamp01(psi[V_FS]);
        double rho_pt = mix(P->rho, Cc, Fs);
        double cp_pt = mix(P->cp, Cc, Fs);
        feq_pt[al] = feq(Q9_W[al], ex, ey, psi[V_P], rho_pt, psi[V_U], psi[V_V]);
        feqm_pt[al] = feqm(Q9_W[al], ex, ey, psi[V_P], rho_f, psi[V_U], psi[V_V]);
        if (al < Qhg) {
            heq_pt[al] = al == 0 ? 0.0 : heq(Whg[al], ex, ey, psi[V_T], cp_pt, cpref, psi[V_U], psi[V_V]);
            geq_pt[al] = geq(al, Whg[al], ex, ey, psi[V_C], psi[V_MUC], P->Qg, psi[V_U], psi[V_V]);
        }
    }

    /* step (3): Eq. (56), the face state at the new level */
    double p_new = 0.0, mx = 0.0, my = 0.0, C_new = 0.0;
    for (int al = 0; al < 9; ++al) {
        p_new += feq_pt[al];
        mx += Q9_EX[al] * feq_pt[al];
        my += Q9_EY[al] * feq_pt[al];
    }
    for (int al = 0; al < Qhg; ++al) C_new += geq_pt[al];
    double u_new = mx / (rho_f * CS2);
    double v_new = my / (rho_f * CS2);

    /* face equilibria */
    double feq_f[9], heq_f[9], geq_f[9];
    for (int al = 0; al < 9; ++al)
        feq_f[al] = feq(Q9_W[al], Q9_EX[al], Q9_EY[al], p_new, rho_f, u_new, v_new);
    for (int al = 0; al < Qhg; ++al) {
        heq_f[al] = al == 0 ? 0.0 : heq(Whg[al], Q9_EX[al], Q9_EY[al], T_f, cp_f, cpref, u_new, v_new);
        geq_f[al] = geq(al, Whg[al], Q9_EX[al], Q9_EY[al], C_new, muc_f, P->Qg, u_new, v_new);
    }

    /* step (1): relaxation parameters at the face */
    double tau_h = 0.5 + lam_f / (rho_f * cpref * CS2 * dt);
    double tau_f = 0.5 + mu_f / (rho_f * CS2 * dt);
    double tau_g = 0.5 + P->mobility / (P->Qg * dt);

    /* step (4): non-equilibrium parts and star distributions; step (5): moments */
    double FH = 0.0, Fp = 0.0, FMx = 0.0, FMy = 0.0, FC = 0.0;
    for (int al = 0; al < 9; ++al) {
        int ex = Q9_EX[al], ey = Q9_EY[al];
        int en = ex * nxn + ey * nyn;
        double fneqm = -tau_f * (feq_f[al] - feqm_pt[al]);            /* Eq. (35) */
        double fstar = feq_f[al] + (1.0 - 1.0 / (2.0 * tau_f)) * fneqm; /* Eq. (37), R2 */
        Fp += en * feq_f[al];
        FMx += en * ex * fstar;
        FMy += en * ey * fstar;
    }
    for (int al = 1; al < Qhg; ++al) {
        int en = Q9_EX[al] * nxn + Q9_EY[al] * nyn;
        double hneq = -tau_h * (heq_f[al] - heq_pt[al]);               /* Eq. (13) */
        double hstar = heq_f[al] + (1.0 - 1.0 / (2.0 * tau_h)) * hneq; /* Eq. (16) */
        double gneq = -tau_g * (geq_f[al] - geq_pt[al]);               /* Eq. (44) */
        double gstar = geq_f[al] + (1.0 - 1.0 / (2.0 * tau_g)) * gneq; /* Eq. (46) */
        FH += en * hstar;
        FC += en * gstar;
    }
    F[0] = FH;
    F[1] = Fp;
    F[2] = FMx;
    F[3] = FMy;
    F[4] = FC;
}

/* R13 flux conditions on a wall face */
static void wall_face(const or_params* P, int side, double F[5])
{
    const or_bc* b = &P->bc[side];
    if (b->periodic) return;
    if (b->flow != OR_FLOW_OUTLET) F[1] = 0.0;
    F[4] = 0.0;
    if (b->heat == OR_HEAT_ADIABATIC) F[0] = 0.0;
}

/* Residual R(W) of Eq. (57) on the interior; W and R are 5 planes of nx*ny
 * (row-major, x fastest).  Fx: 5 planes of (nx+1)*ny (face i on the left of
 * column i), Fy: 5 planes of nx*(ny+1) (face j below row j); either may be
 * NULL. */
static void residual(grid_t* g, const double* Fsdot, double* R, double* Fx, double* Fy)
{
    const or_params* P = g->P;
    int nx = g->nx, ny = g->ny;
    size_t nfx = (size_t)(nx + 1) * ny, nfy = (size_t)nx * (ny + 1), nc = (size_t)nx * ny;
    double* fx = (double*)malloc(5 * nfx * sizeof(double));
    double* fy = (double*)malloc(5 * nfy * sizeof(double));
    fill_ghosts(g);
    derive_all(g);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i <= nx; ++i) {
            double F[5];
            face_flux(P, at(g, i - 1, j), at(g, i, j), 0, 0.5 * WX(g, i - 1), 0.5 * WX(g, i), F);
            if (i == 0) wall_face(P, 0, F);
            if (i == nx) wall_face(P, 1, F);
            for (int k = 0; k < 5; ++k) fx[k * nfx + (size_t)j * (nx + 1) + i] = F[k];
        }
#pragma omp parallel for schedule(static)
    for (int j = 0; j <= ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double F[5];
            face_flux(P, at(g, i, j - 1), at(g, i, j), 1, 0.5 * WY(g, j - 1), 0.5 * WY(g, j), F);
            if (j == 0) wall_face(P, 2, F);
            if (j == ny) wall_face(P, 3, F);
            for (int k = 0; k < 5; ++k) fy[k * nfy + (size_t)j * nx + i] = F[k];
        }
    const double ratio = P->rho[0] / P->rho[1]; /* rho_s / rho_l */
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const cell_t* c = at(g, i, j);
            double fs_dot = Fsdot ? Fsdot[(size_t)j * nx + i] : 0.0;
            double u = c->val[V_U], v = c->val[V_V], C = c->W[4];
            double div_u = c->grad[V_U][0] + c->grad[V_V][1];
            double drho_x = d1(HXM(g, i), HXP(g, i), at(g, i - 1, j)->rho, c->rho, at(g, i + 1, j)->rho);
            double drho_y = d1(HYM(g, j), HYP(g, j), at(g, i, j - 1)->rho, c->rho, at(g, i, j + 1)->rho);
            double surf = P->surf_model == 1 ? -c->Fl * C : -C; /* F_surf = surf * grad mu_c */
            double S[5];
            S[0] = c->cp * c->val[V_T] * div_u;                                   /* Eq. 51 row 1 */
            S[1] = (u * drho_x + v * drho_y) * CS2 + c->rho * CS2 * (1.0 - ratio) * fs_dot; /* row 2 */
            S[2] = CS2 * (surf * c->grad[V_MUC][0] - c->rho * u * fs_dot + c->rho * P->gx);  /* row 3 */
            S[3] = CS2 * (surf * c->grad[V_MUC][1] - c->rho * v * fs_dot + c->rho * P->gy);  /* row 4 */
            S[4] = (P->c_source == 1 ? C * (1.0 - ratio) : (1.0 - ratio)) * fs_dot; /* R5 */
            for (int k = 0; k < 5; ++k) {
                double dfx = fx[k * nfx + (size_t)j * (nx + 1) + i + 1] - fx[k * nfx + (size_t)j * (nx + 1) + i];
                double dfy = fy[k * nfy + (size_t)(j + 1) * nx + i] - fy[k * nfy + (size_t)j * nx + i];
                /* Eq. (52) on a Cartesian cell: V = w_i h_j, S = h_j (x faces), w_i (y faces) */
                R[k * nc + (size_t)j * nx + i] = -dfx / WX(g, i) - dfy / WY(g, j) + S[k];
            }
        }
    if (Fx) memcpy(Fx, fx, 5 * nfx * sizeof(double));
    if (Fy) memcpy(Fy, fy, 5 * nfy * sizeof(double));
    free(fx);
    free(fy);
}

static double solid_fraction(const or_params* P, double H, double C)
{
    double Fl, T;
    or_closure(P, H, C, &Fl, &T);
    return clamp01(C) * (1.0 - Fl);
}

/* R12: momentum projection after a stage */
static void project(const or_params* P, double* W)
{
    size_t n = (size_t)P->nx * P->ny;
    for (size_t q = 0; q < n; ++q) {
        double Fs = solid_fraction(P, W[q], W[4 * n + q]);
        W[2 * n + q] *= (1.0 - Fs);
        W[3 * n + q] *= (1.0 - Fs);
    }
}

/* ---------------------------------------------------------------------------
 * Public entry points.
 * ------------------------------------------------------------------------- */
/* smallest width of n cells (dx where the array is NULL); 0 if one is not a
 * finite positive number */
static double min_width(const double* w, double dx, int n)
{
    if (!w) return dx;
    double m = w[0];
    for (int i = 0; i < n; ++i) {
        if (!(w[i] > 0.0) || !isfinite(w[i])) return 0.0;
        if (w[i] < m) m = w[i];
    }
    return m;
}

static int check(const or_params* P)
{
    if (!P || P->nx < 1 || P->ny < 1 || P->dx <= 0.0) return OR_EINVAL;
    double wmin = fmin(min_width(P->xw, P->dx, P->nx), min_width(P->yw, P->dx, P->ny));
    if (!(wmin > 0.0)) return OR_EINVAL;
    if (P->delta_t <= 0.0 || P->delta_t > 0.5 * wmin * (1.0 + 1e-15)) return OR_EINVAL;
    if (P->lattice_hg != 5 && P->lattice_hg != 9) return OR_EINVAL;
    if (P->c_source != 0 && P->c_source != 1) return OR_EINVAL;
    if (P->bc[0].periodic != P->bc[1].periodic || P->bc[2].periodic != P->bc[3].periodic) return OR_EINVAL;
    if (!P->bc[0].periodic && P->nx < NG) return OR_EINVAL;
    if (!P->bc[2].periodic && P->ny < NG) return OR_EINVAL;
    for (int s = 0; s < 4; ++s) {
        const or_bc* b = &P->bc[s];
        if (b->theta_adv == 0.0 && b->theta_rec == 0.0) continue;
        if (!(b->theta_rec > 0.0 && b->theta_rec <= b->theta_deg && b->theta_deg <= b->theta_adv &&
              b->theta_adv < 180.0))
            return OR_EINVAL;
    }
    return OR_OK;
}

int or_init(const or_params* P, const double* T, const double* Fl, const double* C, const double* u,
            const double* v, const double* p, double* W)
{
    if (check(P)) return OR_EINVAL;
    size_t n = (size_t)P->nx * P->ny;
    for (size_t q = 0; q < n; ++q) {
        double H = enthalpy_of(P, T[q], Fl[q], C[q]);
        double Fs = solid_fraction(P, H, C[q]);
        double Cc = clamp01(C[q]);
        double rho = mix(P->rho, Cc, Fs);
        W[q] = H;
        W[n + q] = p[q];
        W[2 * n + q] = rho * CS2 * u[q];
        W[3 * n + q] = rho * CS2 * v[q];
        W[4 * n + q] = C[q];
    }
    return OR_OK;
}

int or_ghosts(const or_params* P, const double* W, double* Wg)
{
    if (check(P)) return OR_EINVAL;
    grid_t g;
    if (grid_alloc(&g, P)) return OR_EINVAL;
    load_interior(&g, W);
    fill_ghosts(&g);
    size_t ng = (size_t)g.sx * (P->ny + 2 * NG);
    for (int j = -NG; j < P->ny + NG; ++j)
        for (int i = -NG; i < P->nx + NG; ++i)
            for (int k = 0; k < 5; ++k) Wg[k * ng + (size_t)(j + NG) * g.sx + (i + NG)] = at(&g, i, j)->W[k];
    grid_free(&g);
    return OR_OK;
}

int or_residual(const or_params* P, const double* W, const double* Fsdot, double* R, double* Fx, double* Fy)
{
    if (check(P)) return OR_EINVAL;
    grid_t g;
    if (grid_alloc(&g, P)) return OR_EINVAL;
    load_interior(&g, W);
    residual(&g, Fsdot, R, Fx, Fy);
    grid_free(&g);
    return OR_OK;
}

/* Eq. (58) with R11 and R12; W (5 planes) and Fsdot (1 plane) advance in place. */
int or_step(const or_params* P, double* W, double* Fsdot, int64_t nsteps)
{
    if (check(P)) return OR_EINVAL;
    size_t n = (size_t)P->nx * P->ny, n5 = 5 * n;
    double* W1 = (double*)malloc(n5 * sizeof(double));
    double* W2 = (double*)malloc(n5 * sizeof(double));
    double* R = (double*)malloc(n5 * sizeof(double));
    double* Fs0 = (double*)malloc(n * sizeof(double));
    grid_t g;
    if (!W1 || !W2 || !R || !Fs0 || grid_alloc(&g, P)) {
        free(W1); free(W2); free(R); free(Fs0);
        return OR_EINVAL;
    }
    const double dt = P->dt;
    for (int64_t s = 0; s < nsteps; ++s) {
        for (size_t q = 0; q < n; ++q) Fs0[q] = solid_fraction(P, W[q], W[4 * n + q]);
        /* W1 = W^n + dt R(W^n) */
        load_interior(&g, W);
        residual(&g, Fsdot, R, NULL, NULL);
        for (size_t q = 0; q < n5; ++q) W1[q] = W[q] + dt * R[q];
        project(P, W1);
        /* W2 = 3/4 W^n + 1/4 W1 + 1/4 dt R(W1) */
        load_interior(&g, W1);
        residual(&g, Fsdot, R, NULL, NULL);
        for (size_t q = 0; q < n5; ++q) W2[q] = 0.75 * W[q] + 0.25 * W1[q] + 0.25 * dt * R[q];
        project(P, W2);
        /* W^{n+1} = 1/3 W^n + 2/3 W2 + 2/3 dt R(W2) */
        load_interior(&g, W2);
        residual(&g, Fsdot, R, NULL, NULL);
        for (size_t q = 0; q < n5; ++q) W[q] = W[q] / 3.0 + 2.0 / 3.0 * W2[q] + 2.0 / 3.0 * dt * R[q];
        project(P, W);
        /* R11: lagged solid-fraction rate for the next step */
        for (size_t q = 0; q < n; ++q) Fsdot[q] = (solid_fraction(P, W[q], W[4 * n + q]) - Fs0[q]) / dt;
    }
    grid_free(&g);
    free(W1); free(W2); free(R); free(Fs0);
    return OR_OK;
}

/* Primitive fields (T, F_l, F_s, rho, u, v, mu_c) of the interior, 7 planes. */
int or_primitives(const or_params* P, const double* W, double* out)
{
    if (check(P)) return OR_EINVAL;
    grid_t g;
    if (grid_alloc(&g, P)) return OR_EINVAL;
    load_interior(&g, W);
    fill_ghosts(&g);
    derive_all(&g);
    size_t n = (size_t)P->nx * P->ny;
    for (int j = 0; j < P->ny; ++j)
        for (int i = 0; i < P->nx; ++i) {
            const cell_t* c = at(&g, i, j);
            size_t q = (size_t)j * P->nx + i;
            out[q] = c->val[V_T];
            out[n + q] = c->Fl;
            out[2 * n + q] = c->Fs;
            out[3 * n + q] = c->rho;
            out[4 * n + q] = c->val[V_U];
            out[5 * n + q] = c->val[V_V];
            out[6 * n + q] = c->val[V_MUC];
        }
    grid_free(&g);
    return OR_OK;
}

/* FP64 integrals: [sum rho dV, sum C dV, sum H dV, sum F_s dV, max |u|] */
int or_diagnostics(const or_params* P, const double* W, double* out)
{
    if (check(P)) return OR_EINVAL;
    size_t n = (size_t)P->nx * P->ny;
    double s_rho = 0, s_c = 0, s_h = 0, s_fs = 0, umax = 0;
    for (size_t q = 0; q < n; ++q) {
        int i = (int)(q % (size_t)P->nx), j = (int)(q / (size_t)P->nx);
        double dV = (P->xw ? P->xw[i] : P->dx) * (P->yw ? P->yw[j] : P->dx); /* R24 */
        double H = W[q], C = W[4 * n + q];
        double Fl, T;
        or_closure(P, H, C, &Fl, &T);
        double Cc = clamp01(C);
        double Fs = Cc * (1.0 - Fl);
        double rho = mix(P->rho, Cc, Fs);
        double u = W[2 * n + q] / (rho * CS2), v = W[3 * n + q] / (rho * CS2);
        s_rho += rho * dV;
        s_c += C * dV;
        s_h += H * dV;
        s_fs += Fs * dV;
        double sp = sqrt(u * u + v * v);
        if (sp > umax) umax = sp;
    }
    out[0] = s_rho;
    out[1] = s_c;
    out[2] = s_h;
    out[3] = s_fs;
    out[4] = umax;
    return OR_OK;
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
