/*
 * FP64 CPU oracle of the EULBFS time step -- TEST INFRASTRUCTURE ONLY.
 *
 * Used by the tests, the smoke check and the CPU-baseline leg of the
 * benchmark; never by the product path.  Shares nothing with the HIP library.
 * Every array is a set of planes, row-major with x fastest: the conserved
 * vector W = (H, p, rho c_s^2 u, rho c_s^2 v, C) of Eq. (49) is 5 planes of
 * nx*ny doubles.  All functions return 0 on success and -1 on bad parameters.
 */
#ifndef EULBFS_ORACLE_H
#define EULBFS_ORACLE_H
#include <stdint.h>

#define OR_OK 0
#define OR_EINVAL -1

enum { OR_FLOW_NOSLIP = 0, OR_FLOW_FREESLIP = 1, OR_FLOW_OUTLET = 2 };
enum { OR_HEAT_ADIABATIC = 0, OR_HEAT_DIRICHLET = 1 };

typedef struct {
    int32_t periodic; /* 1: periodic in this direction (both sides must agree) */
    int32_t flow;     /* OR_FLOW_* for a wall */
    int32_t heat;     /* OR_HEAT_* for a wall */
    int32_t pad;
    double T_w;       /* wall temperature for OR_HEAT_DIRICHLET */
    double theta_deg; /* contact angle; 90 = plain no-flux wall */
    double theta_adv, theta_rec; /* hysteresis window (R23); 0, 0: none */
} or_bc;

typedef struct {
    int32_t nx, ny;
    int32_t lattice_hg; /* 9 (paper) or 5: lattice of h and g; f is always D2Q9 */
    int32_t surf_model; /* 0: F_surf = -C grad mu_c; 1: -F_l C grad mu_c */
    int32_t c_source;   /* C source (R5): 0: (1 - r) dF_s/dt; 1: C (1 - r) dF_s/dt */
    int32_t pad;
    double dx;
    double delta_t; /* streaming step, 0 < delta_t <= dx/2 */
    double dt;      /* update step of the RK3 scheme */
    double rho[3], mu[3], lam[3], cp[3]; /* solid, liquid, gas (Eq. 7) */
    double latent, T_s, T_l;
    double sigma, xi, mobility, Qg;
    double gx, gy;
    or_bc bc[4]; /* x-, x+, y-, y+ */
    /* Stretched mesh (R24): nx column widths and ny row heights, or NULL for
     * the uniform spacing dx in that direction. */
    const double* xw;
    const double* yw;
} or_params;

void or_closure(const or_params* P, double H, double C, double* Fl, double* T);
void or_equilibria(const or_params* P, double H, double T, double cp, double p, double rho,
                   double C, double muc, double u, double v, double* h_out, double* f_out,
                   double* g_out);
int or_init(const or_params* P, const double* T, const double* Fl, const double* C,
            const double* u, const double* v, const double* p, double* W);
int or_ghosts(const or_params* P, const double* W, double* Wg);
int or_residual(const or_params* P, const double* W, const double* Fsdot, double* R, double* Fx,
                double* Fy);
int or_step(const or_params* P, double* W, double* Fsdot, int64_t nsteps);
int or_primitives(const or_params* P, const double* W, double* out);
int or_diagnostics(const or_params* P, const double* W, double* out);
int or_num_threads(void);
void or_set_threads(int n);

#endif
