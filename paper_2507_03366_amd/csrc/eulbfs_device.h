// Device-side building blocks of the EULBFS time step for gfx950.
//
// Everything here is templated on the field/arithmetic type R (double or
// float).  Two fields are always stored and combined in double: the total
// enthalpy H, whose closure H -> (T, F_l) of Eqs. (5)-(6) also runs in double
// (in FP32 mode the enthalpy increments per step are far below the float
// spacing of H ~ L near the melting point), and the order parameter C, whose
// chemical potential 2 beta C(C-1)(2C-1) - kappa lap C is a difference of two
// nearly equal terms across the diffuse interface (a float C puts a noise of
// ~1e-8 on the capillary force that drives p and u).
//
// Storage: structure of arrays.  Each conserved field is one plane of
// ny rows of `pitch` elements (pitch >= nx, a multiple of 64), x fastest.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace eulbfs {

constexpr int NG = 3;  // ghost layers needed by the stencil (C -> mu_c -> grad -> face)

enum { FLOW_NOSLIP = 0, FLOW_FREESLIP = 1, FLOW_OUTLET = 2 };
enum { HEAT_ADIABATIC = 0, HEAT_DIRICHLET = 1 };

// Constants of one problem, derived on the host once (passed by value as a
// kernel argument).
struct DevParams {
    int nx, ny, pitch;
    int lattice_hg;   // 9 or 5 (h and g); the flow lattice is always D2Q9
    int surf_model;   // 0: -C grad mu_c, 1: -F_l C grad mu_c
    int c_source;     // C source: 0: (1 - r) dF_s/dt, 1: C (1 - r) dF_s/dt
    int periodic_x, periodic_y;
    int flow[4], heat[4];
    double dx, inv_dx, inv_2dx, inv_dx2, delta_t, dt;
    double rho[3], mu[3], lam[3], cp[3];  // solid, liquid, gas (Eq. 7)
    double latent, T_s, T_l;
    double beta, kappa;  // 12 sigma/xi, 3 xi sigma/2 (Sec. 2.3.1)
    double a_g;          // tau_g - 1/2 = M_c / (Q_g delta_t)   (Eq. 41)
    double muQ;          // Q_g
    double cpref;        // (C_p,s + C_p,l)/2                   (Sec. 2.1.2)
    double k_h;          // 3 / (C_p,ref delta_t): tau_h - 1/2 = k_h lambda/rho
    double k_f;          // 3 / delta_t:           tau_f - 1/2 = k_f mu/rho
    double gx, gy;
    double expansion;    // 1 - rho_s/rho_l
    double T_w[4];
    double wet[4];       // dx (4/xi) cos(theta): ghost C offset per mirror distance
    double wet_k;        // dx (4/xi)
    int hyst[4];         // contact-angle hysteresis window on this wall
    double cos_adv[4], cos_rec[4];  // cos of the advancing and receding angles
    double inv_dt;
    double half_off[2];  // FAST_HALF point offsets of the stored differences: 1/4 (cells), 1/8 (face)
    int fast;            // FAST_* fast paths valid for these constants
    // FAST_UCP closure constants: H_s = C_p T_s, H_l = C_p T_l + L, 1/C_p,
    // 1/(H_l - H_s) (0 without a mushy range)
    double Hs_u, Hl_u, inv_cp, inv_dH;
    // Stretched tensor-product mesh (the NU variants of the kernels); all
    // NULL on a uniform mesh.  mside: per side, MS_STRIDE doubles (MS_*).  mxc, myc:
    // NMESH arrays (MESH_*) over the ghosted columns / rows, msx / msy apart.
    const double* mside;
    const double* mxc;
    const double* myc;
    int msx, msy;
};

// Per-cell mesh coefficients along one direction, at ghosted index l:
//   MESH_GM, MESH_G0, MESH_GP  d psi/ds = GM psi_{l-1} + G0 psi_l + GP psi_{l+1}
//                              (derivative of the parabola through the three
//                              centres; (psi_{l+1} - psi_{l-1}) / (2 dx) when uniform)
//   MESH_LM, MESH_L0, MESH_LP  d2 psi/ds2 of the same parabola
//   MESH_HW                    half width of the cell
//   MESH_IW                    1 / width
enum { MESH_GM = 0, MESH_G0, MESH_GP, MESH_LM, MESH_L0, MESH_LP, MESH_HW, MESH_IW, NMESH };
// Per wall side: MS_D + k - 1 distance between the centres of ghost layer k
// and its mirror cell; MS_L0..2 weights of dC/dn at the wall from the first
// three interior cells; MS_WET (4/xi) cos(theta); MS_K 4/xi.
enum { MS_D = 0, MS_L0 = 3, MS_WET = 6, MS_K = 7, MS_STRIDE = 8 };

// Fast paths compiled as template flags.  Each computes the same quantities
// as the general code (equal up to rounding order), with fewer operations:
//  FAST_HALF  delta_t = dx/2: the surrounding points with e_n = +-1, e_t = 0
//             are the two cell centres, so no extrapolation along n is
//             needed there and their density is the cell's; the face value
//             is 5/8 (psi_a + psi_b) - 1/8 (psi_a-1 + psi_b+1), and the
//             tangential differences are kept unscaled with their factor
//             (1/4, or 1/8 for the face group) folded into the coefficients.
//  FAST_UCP   one heat capacity for all phases: every Eq. (7) mixture of C_p
//             is that constant, and the closure's H_s, H_l and reciprocals
//             are constants of the run.
enum { FAST_HALF = 1, FAST_UCP = 2 };

// Pointers to one copy of the conserved vector W = (H, p, Mx, My, C).
template <typename R>
struct State {
    double* H;
    R* p;
    R* mx;
    R* my;
    double* C;
};

template <typename R>
struct Cons {
    double H;
    R p, mx, my;
    double C;
};

__device__ __forceinline__ double clamp01(double x) { return fmin(fmax(x, 0.0), 1.0); }
__device__ __forceinline__ float clamp01(float x) { return fminf(fmaxf(x, 0.0f), 1.0f); }

// 1/x from the hardware reciprocal estimate refined by two Newton steps
// (within an ulp or two of the correctly rounded value for the positive,
// normal operands used here: densities, heat capacities, enthalpy ranges).
__device__ __forceinline__ double rcp(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Eq. (7): gamma = F_s g_s + (1 - F_s) C g_l + (1 - F_s)(1 - C) g_g.
template <typename R>
__device__ __forceinline__ R mix(const double g[3], R C, R Fs)
{
    const R gs = R(g[0]), gl = R(g[1]), gg = R(g[2]);
    const R cond = gg + C * (gl - gg);  // C g_l + (1 - C) g_g
    return cond + Fs * (gs - cond);
}

// Eqs. (5)-(6) with H = C_p T + L F_l and the condensed-phase mixtures
// C_p^S = Eq.7(C, F_s = C), C_p^L = Eq.7(C, F_s = 0).  Cc is C clamped to [0,1].
template <int FAST = 0>
__device__ __forceinline__ void closure(const DevParams& P, double H, double Cc, double& Fl, double& T)
{
    if (FAST & FAST_UCP) {  // one C_p: H_s, H_l and the reciprocals are constants
        if (H < P.Hs_u) {
            Fl = 0.0;
            T = P.T_s + (H - P.Hs_u) * P.inv_cp;
        } else if (H > P.Hl_u) {
            Fl = 1.0;
            T = P.T_l + (H - P.Hl_u) * P.inv_cp;
        } else {
            Fl = P.inv_dH > 0.0 ? (H - P.Hs_u) * P.inv_dH : 1.0;
            T = P.T_s + Fl * (P.T_l - P.T_s);
        }
        return;
    }
    const double cpS = mix<double>(P.cp, Cc, Cc);
    const double cpL = mix<double>(P.cp, Cc, 0.0);
    const double Hs = cpS * P.T_s;
    const double Hl = cpL * P.T_l + P.latent;
    if (H < Hs) {
        Fl = 0.0;
        T = P.T_s + (H - Hs) * rcp(cpS);
    } else if (H > Hl) {
        Fl = 1.0;
        T = P.T_l + (H - Hl) * rcp(cpL);
    } else {
        const double d = Hl - Hs;
        Fl = d > 1e-300 ? (H - Hs) * rcp(d) : 1.0;
        T = P.T_s + Fl * (P.T_l - P.T_s);
    }
}

template <int FAST = 0>
__device__ __forceinline__ double solid_fraction(const DevParams& P, double H, double C)
{
    const double Cc = clamp01(C);
    double Fl, T;
    closure<FAST>(P, H, Cc, Fl, T);
    return Cc * (1.0 - Fl);
}

// Enthalpy of a state with temperature T and liquid fraction Fl.
__device__ __forceinline__ double enthalpy_of(const DevParams& P, double T, double Fl, double C)
{
    const double Cc = clamp01(C);
    const double cpS = mix<double>(P.cp, Cc, Cc);
    const double cpL = mix<double>(P.cp, Cc, 0.0);
    const double Hs = cpS * P.T_s;
    const double Hl = cpL * P.T_l + P.latent;
    return (1.0 - Fl) * (Hs + cpS * (T - P.T_s)) + Fl * (Hl + cpL * (T - P.T_l));
}

// Inverse closure for a Dirichlet ghost cell: phase from T against T_s, T_l.
__device__ __forceinline__ double ghost_enthalpy(const DevParams& P, double T, double C)
{
    double Fl;
    if (T > P.T_l)
        Fl = 1.0;
    else if (T < P.T_s)
        Fl = 0.0;
    else if (P.T_l > P.T_s)
        Fl = (T - P.T_s) / (P.T_l - P.T_s);
    else
        Fl = 1.0;
    return enthalpy_of(P, T, Fl, C);
}

// Conserved state of the cell at linear index q = j * pitch + i.
template <typename R>
__device__ __forceinline__ Cons<R> read_at(const State<R>& S, size_t q)
{
    Cons<R> w;
    w.H = S.H[q];
    w.p = S.p[q];
    w.mx = S.mx[q];
    w.my = S.my[q];
    w.C = S.C[q];
    return w;
}

template <typename R>
__device__ __forceinline__ Cons<R> read_cell(const State<R>& S, int pitch, int i, int j)
{
    const size_t q = (size_t)j * pitch + i;
    Cons<R> w;
    w.H = S.H[q];
    w.p = S.p[q];
    w.mx = S.mx[q];
    w.my = S.my[q];
    w.C = S.C[q];
    return w;
}

// Wetting factor dx (4/xi) cos(theta) of a wall.  With a hysteresis window the
// angle is the apparent one of the first three interior cells along the
// inward normal (C1, C2, C3), cos = -dC/dn / ((4/xi) C1 (1 - C1)) with dC/dn at
// the wall from the quadratic through the three cell centres, clamped to the
// window; where C1 (1 - C1) <= 1e-3 there is no interface and the equilibrium
// angle is used.
__device__ __forceinline__ double wet_factor(const DevParams& P, int side, double C1, double C2, double C3)
{
    const double s = C1 * (1.0 - C1);
    if (!P.hyst[side] || !(s > 1e-3)) return P.wet[side];
    const double dn = -2.0 * C1 + 3.0 * C2 - C3;
    const double c = fmin(fmax(-dn / (P.wet_k * s), P.cos_adv[side]), P.cos_rec[side]);
    return P.wet_k * c;
}

// Stretched mesh: (4/xi) cos(theta) of a wall, the apparent angle read from
// the first three interior cells with the side's own weights when the wall
// has a hysteresis window (same rule as wet_factor).
__device__ __forceinline__ double wet_factor_nu(const DevParams& P, int side, double C1, double C2, double C3)
{
    const double* ms = P.mside + side * MS_STRIDE;
    const double s = C1 * (1.0 - C1);
    if (!P.hyst[side] || !(s > 1e-3)) return ms[MS_WET];
    const double dn = ms[MS_L0] * C1 + ms[MS_L0 + 1] * C2 + ms[MS_L0 + 2] * C3;
    const double c = fmin(fmax(-dn / (ms[MS_K] * s), P.cos_adv[side]), P.cos_rec[side]);
    return ms[MS_K] * c;
}

// Wall rule for ghost layer k (1..3) of `side` (0 x-, 1 x+, 2 y-, 3 y+):
// m is the mirrored interior cell, Cw the C of the first interior cell, wet
// the wall's wetting factor (wet_factor; wet_factor_nu on a stretched mesh,
// NU, where the ghost-to-mirror distance comes from the side's table).
template <typename R, bool NU = false>
__device__ __forceinline__ Cons<R> wall_ghost(const DevParams& P, int side, int k, const Cons<R>& m, double Cw,
                                              double wet)
{
    Cons<R> g;
    g.p = m.p;
    const bool xside = side < 2;
    const R mn = xside ? m.mx : m.my;
    const R mt = xside ? m.my : m.mx;
    const int f = P.flow[side];
    const R gn = f == FLOW_OUTLET ? mn : -mn;
    const R gt = f == FLOW_NOSLIP ? -mt : mt;
    g.mx = xside ? gn : gt;
    g.my = xside ? gt : gn;
    if (NU)
        g.C = m.C + (P.mside[side * MS_STRIDE + MS_D + k - 1] * wet) * Cw * (1.0 - Cw);
    else
        g.C = m.C + ((2 * k - 1) * wet) * Cw * (1.0 - Cw);
    if (P.heat[side] == HEAT_DIRICHLET) {
        double Fl, Tm;
        closure(P, m.H, clamp01(m.C), Fl, Tm);
        const double Tg = 2.0 * P.T_w[side] - Tm;
        g.H = ghost_enthalpy(P, Tg, g.C);
    } else {
        g.H = m.H;
    }
    return g;
}

__device__ __forceinline__ int wrap(int i, int n)
{
    int r = i % n;
    return r < 0 ? r + n : r;
}

// Conserved state at (i, j) for j inside [0, ny): interior read, periodic copy
// or x-wall rule (NU: stretched-mesh wall geometry).
template <typename R, bool NU = false>
__device__ __forceinline__ Cons<R> load_x(const DevParams& P, const State<R>& S, int i, int j)
{
    if (i >= 0 && i < P.nx) return read_cell(S, P.pitch, i, j);
    if (P.periodic_x) return read_cell(S, P.pitch, wrap(i, P.nx), j);
    int side, k, m, first, in;
    if (i < 0) {
        side = 0; k = -i; m = k - 1; first = 0; in = 1;
    } else {
        side = 1; k = i - P.nx + 1; m = P.nx - k; first = P.nx - 1; in = -1;
    }
    const Cons<R> wm = read_cell(S, P.pitch, m, j);
    const size_t o = (size_t)j * P.pitch + first;
    const double Cw = S.C[o];
    double wet;
    if (NU)
        wet = P.hyst[side] ? wet_factor_nu(P, side, Cw, S.C[o + in], S.C[o + 2 * in])
                           : P.mside[side * MS_STRIDE + MS_WET];
    else
        wet = P.hyst[side] ? wet_factor(P, side, Cw, S.C[o + in], S.C[o + 2 * in]) : P.wet[side];
    return wall_ghost<R, NU>(P, side, k, wm, Cw, wet);
}

// Conserved state at any (i, j) of the grid extended by the three-layer
// ghost ring: x rule on the interior rows, then the y rule on every column
// (corner cells take the y rule of x-ghost cells).  Indices beyond the ring
// are clamped onto it (only partial edge tiles reach them; their results are
// never stored).  NU: stretched-mesh wall geometry.
template <typename R, bool NU = false>
__device__ __forceinline__ Cons<R> load_bc(const DevParams& P, const State<R>& S, int i, int j)
{
    i = min(max(i, -NG), P.nx + NG - 1);
    j = min(max(j, -NG), P.ny + NG - 1);
    if (j >= 0 && j < P.ny) return load_x<R, NU>(P, S, i, j);
    if (P.periodic_y) return load_x<R, NU>(P, S, i, wrap(j, P.ny));
    int side, k, m, first, in;
    if (j < 0) {
        side = 2; k = -j; m = k - 1; first = 0; in = 1;
    } else {
        side = 3; k = j - P.ny + 1; m = P.ny - k; first = P.ny - 1; in = -1;
    }
    const Cons<R> wm = load_x<R, NU>(P, S, i, m);
    const double Cw = load_x<R, NU>(P, S, i, first).C;
    double wet;
    if (NU)
        wet = P.hyst[side] ? wet_factor_nu(P, side, Cw, load_x<R, NU>(P, S, i, first + in).C,
                                           load_x<R, NU>(P, S, i, first + 2 * in).C)
                           : P.mside[side * MS_STRIDE + MS_WET];
    else
        wet = P.hyst[side] ? wet_factor(P, side, Cw, load_x(P, S, i, first + in).C,
                                        load_x(P, S, i, first + 2 * in).C)
                           : P.wet[side];
    return wall_ghost<R, NU>(P, side, k, wm, Cw, wet);
}

// Primitive record of one cell used by the face fluxes.
enum { VT = 0, VC, VFS, VU, VV, VP, VMU, NPRIM };  // + rho stored after

// Closure, Eq. (7) density and velocity of one cell (mu_c done separately).
template <typename R, int FAST = 0>
__device__ __forceinline__ void primitives(const DevParams& P, const Cons<R>& w, R out[NPRIM + 1])
{
    const double Cc = clamp01(w.C);
    double Fl, T;
    closure<FAST>(P, w.H, Cc, Fl, T);
    const R Fs = R(Cc * (1.0 - Fl));
    const R rho = mix<R>(P.rho, R(Cc), Fs);
    const R inv = R(3) * rcp(rho);  // 1 / (rho c_s^2)
    out[VT] = R(T);
    out[VC] = R(w.C);
    out[VFS] = Fs;
    out[VU] = w.mx * inv;
    out[VV] = w.my * inv;
    out[VP] = w.p;
    out[VMU] = R(0);
    out[NPRIM] = rho;
}

// Chemical potential (Sec. 2.3.1): 2 beta C (C-1)(2C-1) - kappa lap C, in
// double whatever the field type.
__device__ __forceinline__ double chem_potential(const DevParams& P, double C, double cE, double cW, double cN,
                                                 double cS)
{
    const double lap = (cE + cW + cN + cS - 4.0 * C) * P.inv_dx2;
    return 2.0 * P.beta * C * (C - 1.0) * (2.0 * C - 1.0) - P.kappa * lap;
}

// The same on a stretched mesh: lap C from the second derivatives of the
// parabolas through the cell (ghosted column li, row lj) and its neighbours.
__device__ __forceinline__ double chem_potential_nu(const DevParams& P, int li, int lj, double C, double cE,
                                                    double cW, double cN, double cS)
{
    const double* mx = P.mxc + li;
    const double* my = P.myc + lj;
    const double lap = mx[MESH_LM * P.msx] * cW + mx[MESH_L0 * P.msx] * C + mx[MESH_LP * P.msx] * cE +
                       my[MESH_LM * P.msy] * cS + my[MESH_L0 * P.msy] * C + my[MESH_LP * P.msy] * cN;
    return 2.0 * P.beta * C * (C - 1.0) * (2.0 * C - 1.0) - P.kappa * lap;
}

// ---------------------------------------------------------------------------
// Face flux (Eqs. 53-56 with Eqs. 9, 13, 16, 29, 33, 35, 37, 42, 44, 46).
//
// Local frame: n is the face normal (from cell a to cell b), t the tangent.
// The D2Q9 set maps onto itself under the x <-> y reflection, so one routine
// serves both orientations: it returns (F_H, F_p, F_Mn, F_Mt, F_C) with
// F_Mn = sum e_n e_n f*, F_Mt = sum e_n e_t f*.
//
// Surrounding points x_f - e delta_t (Eq. 54): e_n = +1 lies in cell a,
// e_n = -1 in cell b, e_n = 0 on the face (average of both extrapolations).
// Every reconstructed value at a point is base - e_t d, with per variable
//   A = psi_a + (dx/2 - delta_t) dpsi_a/dn        (group e_n = +1)
//   B = psi_b - (dx/2 - delta_t) dpsi_b/dn        (group e_n = -1)
//   M = average of both extrapolations to x_f     (group e_n = 0; also the
//                                                  old-level face value)
//   d = delta_t dpsi/dt of the group's cell (the mean for the face group;
//       FAST_HALF keeps 4 d for the cells and 8 d for the face group).
// With a_X = tau_X - 1/2 each star distribution is
//   X* = (1 - a_X) X^eq(x_f) + a_X X^eq(x_f - e delta_t),
// so each flux is (1 - a_X) times a moment of the face equilibrium (closed
// form from Eqs. 11, 29, 42) plus a_X times the same moment of the point
// equilibria.  In those point moments every term that is linear in the
// reconstructed values sums in closed form over the nine points (the
// offsets +-d cancel); only the products rho q, C_p T q and C e.u, with
//   q = e.u/c_s^2 + (e.u)^2/(2 c_s^4) - u^2/(2 c_s^2),
// are evaluated point by point.
// ---------------------------------------------------------------------------
template <typename R>
struct Bases {
    R A[NPRIM], B[NPRIM], M[NPRIM], da[NPRIM], db[NPRIM], dm[NPRIM];
    R rho_a, rho_b;  // cell densities (used by FAST_HALF)
};

// Bases of one variable from a plane of cell values: a and b are the two
// cells (b = a + sn), sn the stride along n, st the stride along t.
template <typename R, int FAST = 0>
__device__ __forceinline__ void face_bases(const R* v, int a, int sn, int st, R c_sh, R c_h, R c_ds, R& A, R& B,
                                           R& M, R& da, R& db, R& dm)
{
    const int b = a + sn;
    const R va = v[a], vb = v[b];
    if (FAST & FAST_HALF) {  // c_sh = 0, c_h = c_ds = 1/4; d kept unscaled
        A = va;
        B = vb;
        M = R(0.625) * (va + vb) - R(0.125) * (v[a - sn] + v[b + sn]);
        da = v[a + st] - v[a - st];
        db = v[b + st] - v[b - st];
        dm = da + db;
        return;
    }
    const R ga = v[b] - v[a - sn];  // 2 dx dpsi_a/dn
    const R gb = v[b + sn] - va;    // 2 dx dpsi_b/dn
    A = va + c_sh * ga;
    B = vb - c_sh * gb;
    M = R(0.5) * ((va + c_h * ga) + (vb - c_h * gb));
    da = c_ds * (v[a + st] - v[a - st]);
    db = c_ds * (v[b + st] - v[b - st]);
    dm = R(0.5) * (da + db);
}

// face_bases on a stretched mesh.  ca, cb: derivative weights (MESH_GM,
// MESH_G0, MESH_GP) along n of cells a and b; ct: those along t of the row
// (column) the face lies in; ha, hb: the two half widths along n; ds:
// delta_t.  A, B, M and d have the meaning stated above, with the true
// derivatives of the two cells.
template <typename R>
__device__ __forceinline__ void face_bases_nu(const R* v, int a, int sn, int st, const R ca[3], const R cb[3],
                                              const R ct[3], R ha, R hb, R ds, R& A, R& B, R& M, R& da, R& db,
                                              R& dm)
{
    const int b = a + sn;
    const R va = v[a], vb = v[b];
    const R ga = ca[0] * v[a - sn] + ca[1] * va + ca[2] * vb;
    const R gb = cb[0] * va + cb[1] * vb + cb[2] * v[b + sn];
    A = va + (ha - ds) * ga;
    B = vb - (hb - ds) * gb;
    M = R(0.5) * ((va + ha * ga) + (vb - hb * gb));
    da = ds * (ct[0] * v[a - st] + ct[1] * va + ct[2] * v[a + st]);
    db = ds * (ct[0] * v[b - st] + ct[1] * vb + ct[2] * v[b + st]);
    dm = R(0.5) * (da + db);
}

template <typename R, int LAT, int FAST = 0>
__device__ __forceinline__ void face_flux(const DevParams& P, const Bases<R>& X, R F[5])
{
    constexpr bool HALF = (FAST & FAST_HALF) != 0, UCP = (FAST & FAST_UCP) != 0;
    // With one C_p and the D2Q9 h lattice the h weights are the f weights, so
    // the point sum of w C_p T q over a group e_n = +-1, with T = T_0 - s e_t d_T
    // at its three points, is C_p (T_0 Q_s - s d_T Q_t) in terms of the sums
    // Q_s = sum w q and Q_t = sum e_t w q the momentum flux needs anyway.
    constexpr bool HQ_SUMS = UCP && LAT == 9;
    // old-level face state (text after Eq. 54) -> Eq. (7)
    const R Cf = clamp01(X.M[VC]);
    const R Fsf = clamp01(X.M[VFS]);
    const R rho_f = mix<R>(P.rho, Cf, Fsf);
    const R mu_f = mix<R>(P.mu, Cf, Fsf);
    const R lam_f = mix<R>(P.lam, Cf, Fsf);
    const R cp_f = UCP ? R(P.cp[0]) : mix<R>(P.cp, Cf, Fsf);

    // point sums: group 0: e_n = +1, group 1: e_n = -1, group 2: e_n = 0
    R G[3] = {0, 0, 0}, Gt[3] = {0, 0, 0};  // sum w rho q, sum e_t w rho q
    R Qs[2] = {0, 0}, Qt[2] = {0, 0};       // sum w q, sum e_t w q      (e_n != 0)
    R Hq[2] = {0, 0};                       // sum wh C_p T q            (e_n != 0)
    R Ce[3] = {0, 0, 0};                    // sum wh C e.u
#pragma unroll
    for (int g = 0; g < 3; ++g) {
        const int en = g == 0 ? 1 : (g == 1 ? -1 : 0);
        const R* base = g == 0 ? X.A : (g == 1 ? X.B : X.M);
        const R* dd = g == 0 ? X.da : (g == 1 ? X.db : X.dm);
        const double dsc = !HALF ? 1.0 : (g == 2 ? 0.125 : 0.25);  // scale of the stored d
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int et = k == 0 ? 0 : (k == 1 ? 1 : -1);
            // FAST_HALF takes the offset scale as a run-time constant: the point
            // value is then one multiply-add with a scalar operand, where a
            // literal 1/4 or 1/8 costs a copy of the base and an accumulate
            // (2 % faster in FP64, the same bits)
            const R ets = HALF ? R(et) * R(P.half_off[g == 2 ? 1 : 0]) : R(et * dsc);
            const R w9 = en == 0 ? (et == 0 ? R(4.0 / 9.0) : R(1.0 / 9.0)) : (et == 0 ? R(1.0 / 9.0) : R(1.0 / 36.0));
            const bool in_hg = LAT == 9 || en == 0 || et == 0;
            const R wh = LAT == 9 ? w9 : (en == 0 && et == 0 ? R(1.0 / 3.0) : R(1.0 / 6.0));
            // e_t = 0: the base itself (0 * d is not folded away in IEEE arithmetic)
            const R C = et == 0 ? base[VC] : base[VC] - ets * dd[VC];
            const R Fs = et == 0 ? base[VFS] : base[VFS] - ets * dd[VFS];
            const R un = et == 0 ? base[VU] : base[VU] - ets * dd[VU];
            const R ut = et == 0 ? base[VV] : base[VV] - ets * dd[VV];
            // a cell centre (HALF, e_n = +-1, e_t = 0) has the cell's density
            const bool centre = HALF && en != 0 && et == 0;
            const R Cc = clamp01(C);
            const R Fsc = clamp01(Fs);
            const R rho = centre ? (g == 0 ? X.rho_a : X.rho_b) : mix<R>(P.rho, Cc, Fsc);
            const R eun = en == 0 ? R(0) : (en > 0 ? un : -un);
            const R eut = et == 0 ? R(0) : (et > 0 ? ut : -ut);
            const R eu = en == 0 ? eut : (et == 0 ? eun : eun + eut);
            const R uu = un * un + ut * ut;
            // q = 3 e.u + 4.5 (e.u)^2 - 1.5 u^2 is carried as q23 = (2/3) q =
            // e.u (2 + 3 e.u) - u^2: two multiply-adds whose constants are an
            // inline 2 and one scalar 3, where 3 and 4.5 together need a copy
            // into registers; the weights of every sum of q carry the 3/2
            const R q23 = eu * (R(2) + R(3) * eu) - uu;
            const R w9q = R(1.5) * w9;
            const R rq = rho * q23;
            G[g] += w9q * rq;
            if (et != 0) Gt[g] += R(et) * w9q * rq;
            if (en != 0) {
                Qs[g] += w9q * q23;
                if (et != 0) Qt[g] += R(et) * w9q * q23;
            }
            if (in_hg) {
                if (en != 0 || et != 0) Ce[g] += wh * C * eu;
                if (en != 0 && !HQ_SUMS) {
                    const R T = et == 0 ? base[VT] : base[VT] - ets * dd[VT];
                    const R cp = UCP ? R(P.cp[0]) : mix<R>(P.cp, Cc, Fsc);
                    Hq[g] += R(1.5) * wh * cp * T * q23;
                }
            }
        }
    }
    const R sixth = R(1.0 / 6.0), third = R(1.0 / 3.0);
    // Eq. (56): new face state from the point equilibria f^eq (Eq. 29) and g^eq (Eq. 42)
    const R p_f = sixth * (X.A[VP] + X.B[VP]) + R(2.0 / 3.0) * X.M[VP] + third * (G[0] + G[1] + G[2]);
    const R m_n = sixth * (X.A[VP] - X.B[VP]) + third * (G[0] - G[1]);
    // with FAST_HALF dm = da + db unscaled: 1/18 (da + db) / 4 + 2/9 dm / 8 = dm / 24
    const R m_t = (HALF ? -R(1.0 / 24.0) * X.dm[VP] : -R(1.0 / 18.0) * (X.da[VP] + X.db[VP]) - R(2.0 / 9.0) * X.dm[VP]) +
                  third * (Gt[0] + Gt[1] + Gt[2]);
    const R Q = R(P.muQ);
    const R C_new = X.M[VC] + R(3) * Q * (sixth * (X.A[VMU] + X.B[VMU]) - third * X.M[VMU]) +
                    R(3) * (Ce[0] + Ce[1] + Ce[2]);
    // point moments of the star distributions (f^eq-m with the face density, Eq. 33)
    const R SMn = sixth * (X.A[VP] + X.B[VP]) + third * rho_f * (Qs[0] + Qs[1]);
    const R SMt = R(HALF ? 1.0 / 72.0 : 1.0 / 18.0) * (X.db[VP] - X.da[VP]) + third * rho_f * (Qt[0] - Qt[1]);
    if constexpr (HQ_SUMS) {
        const R s0 = HALF ? R(P.half_off[0]) : R(1);  // offset scale of the stored d, groups e_n = +-1
        Hq[0] = R(P.cp[0]) * (X.A[VT] * Qs[0] - s0 * (X.da[VT] * Qt[0]));
        Hq[1] = R(P.cp[0]) * (X.B[VT] * Qs[1] - s0 * (X.db[VT] * Qt[1]));
    }
    const R SH = R(P.cpref) * sixth * (X.A[VT] - X.B[VT]) + (Hq[0] - Hq[1]);
    const R SG = R(3) * Q * sixth * (X.A[VMU] - X.B[VMU]) + R(3) * (Ce[0] - Ce[1]);

    const R inv_rho = rcp(rho_f);
    const R un_f = R(3) * m_n * inv_rho;
    const R ut_f = R(3) * m_t * inv_rho;
    const R a_h = R(P.k_h) * lam_f * inv_rho;
    const R a_f = R(P.k_f) * mu_f * inv_rho;
    const R a_g = R(P.a_g);
    F[0] = (R(1) - a_h) * cp_f * X.M[VT] * un_f + a_h * SH;
    F[1] = m_n;
    F[2] = (R(1) - a_f) * (p_f + rho_f * un_f * un_f) * third + a_f * SMn;
    F[3] = (R(1) - a_f) * rho_f * un_f * ut_f * third + a_f * SMt;
    F[4] = (R(1) - a_g) * C_new * un_f + a_g * SG;
}

// Wall-face conditions: no mass flux through an impermeable wall, no
// phase-field flux, no heat flux through an adiabatic wall.
template <typename R>
__device__ __forceinline__ void wall_face(const DevParams& P, int side, R F[5])
{
    if (P.flow[side] != FLOW_OUTLET) F[1] = R(0);
    F[4] = R(0);
    if (P.heat[side] == HEAT_ADIABATIC) F[0] = R(0);
}

// Source vector F_E of Eq. (51) (with the C source in row 5) at one cell.
// c: the cell's primitives (with rho at NPRIM), dux.. central differences.
template <typename R, int FAST = 0>
__device__ __forceinline__ void sources(const DevParams& P, const R c[NPRIM + 1], R Fl, R fsdot, R dudx,
                                        R dvdy, R drhodx, R drhody, R dmudx, R dmudy, R S[5])
{
    const R rho = c[NPRIM];
    const R u = c[VU], v = c[VV], C = c[VC];
    const R cp = (FAST & FAST_UCP) ? R(P.cp[0]) : mix<R>(P.cp, clamp01(C), c[VFS]);
    const R ex = R(P.expansion);
    const R surf = P.surf_model == 1 ? -Fl * C : -C;
    S[0] = cp * c[VT] * (dudx + dvdy);
    S[1] = (u * drhodx + v * drhody) * R(1.0 / 3.0) + rho * R(1.0 / 3.0) * ex * fsdot;
    S[2] = R(1.0 / 3.0) * (surf * dmudx - rho * u * fsdot + rho * R(P.gx));
    S[3] = R(1.0 / 3.0) * (surf * dmudy - rho * v * fsdot + rho * R(P.gy));
    S[4] = (P.c_source ? C * ex : ex) * fsdot;
}

}  // namespace eulbfs
