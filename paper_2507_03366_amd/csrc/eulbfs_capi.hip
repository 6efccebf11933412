// C-ABI runtime of the EULBFS library: parameter validation, workspace
// layout, stage sequencing on the caller's stream, queries and checkpoints.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstddef>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/eulbfs.h"
#include "eulbfs_internal.h"

using namespace eulbfs;

namespace {

thread_local std::string g_thread_err;

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }
inline int round_pitch(int n) { return (n + 63) / 64 * 64; }

int set_err(std::string* where, int code, const std::string& msg)
{
    if (where) *where = msg;
    g_thread_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                                   \
    do {                                                                                                \
        hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess)                                                                           \
            return set_err(err, EULBFS_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));     \
    } while (0)

bool stretched(const eulbfs_params* p) { return p->x_width != nullptr || p->y_width != nullptr; }

// Scratch of eulbfs_residual_noalloc: one array on every device the library
// runs on, held until the process ends.  In host code the name `scratch` is a
// host-side stand-in, not a device address: host code only ever uses the
// per-device address that hipGetSymbolAddress returns (noalloc_scratch).
static __device__ __align__(256) char scratch[EULBFS_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on device dev (which must be current), looked up
// once per device.
int noalloc_scratch(int dev, char** out, std::string* err)
{
    if (dev < 0 || dev >= MAX_DEVICES) return set_err(err, EULBFS_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_err(err, EULBFS_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = (char*)p;
    }
    *out = g_scratch_ptr[dev];
    return EULBFS_OK;
}

// Smallest of n widths (dx for a NULL array); 0 if one is not finite and > 0.
double min_width(const double* w, double dx, int n)
{
    if (!w) return dx;
    double m = w[0];
    for (int i = 0; i < n; ++i) {
        if (!(w[i] > 0) || !std::isfinite(w[i])) return 0.0;
        m = std::min(m, w[i]);
    }
    return m;
}

// Largest eigenvalue of the compact diffusion operator along one direction
// for a unit diffusivity: the finite-volume Laplacian over cells of widths w
// (NULL: n cells of dx) with the distance between neighbouring centres the
// mean of their widths, and at each wall either a mirrored ghost (zero flux)
// or an odd one (a held value at the wall: Dirichlet temperature, no-slip
// momentum).  Its symmetric tridiagonal form is bisected with Sturm counts; a
// periodic direction takes the Gershgorin bound (exact for a uniform mesh of
// even n).
double diffusion_radius(const double* w, double dx, int n, bool periodic, bool odd_lo, bool odd_hi)
{
    auto W = [&](int i) { return w ? w[i] : dx; };
    std::vector<double> a(n, 0.0), b(n, 0.0);  // b[i] couples cells i and i + 1 (mod n)
    for (int i = 0; i < n; ++i) {
        if (i > 0 || periodic) {
            const int j = (i + n - 1) % n;
            a[i] += 1.0 / (W(i) * 0.5 * (W(i) + W(j)));
        } else if (odd_lo) {
            a[i] += 2.0 / (W(i) * W(i));
        }
        if (i < n - 1 || periodic) {
            const int j = (i + 1) % n;
            const double h = 0.5 * (W(i) + W(j));
            a[i] += 1.0 / (W(i) * h);
            b[i] = 1.0 / (h * std::sqrt(W(i) * W(j)));
        } else if (odd_hi) {
            a[i] += 2.0 / (W(i) * W(i));
        }
    }
    double gersh = 0.0;
    for (int i = 0; i < n; ++i) {
        const double left = (i > 0 || periodic) ? b[(i + n - 1) % n] : 0.0;
        gersh = std::max(gersh, a[i] + left + b[i]);
    }
    if (periodic) return gersh;
    double lo = 0.0, hi = gersh;
    for (int it = 0; it < 64; ++it) {
        const double x = 0.5 * (lo + hi);
        int below = 0;  // eigenvalues below x
        double d = 1.0;
        for (int i = 0; i < n; ++i) {
            d = (a[i] - x) - (i > 0 ? b[i - 1] * b[i - 1] / d : 0.0);
            if (d == 0.0) d = -1e-300;
            if (d < 0.0) ++below;
        }
        if (below == n) hi = x;
        else lo = x;
    }
    return hi;
}

// Explicit-step limits of the SSP-RK3 update (Eq. 58) with the fixed dt.  The
// scheme is stable for eigenvalues of the linearised residual down to -2.51 on
// the negative real axis and within sqrt(3) along the imaginary axis.  On the
// compact stencils the fluxes reduce to (Sec. 2.4), a diffusivity D along both
// directions has eigenvalues down to -D (lx + ly), lx and ly the radii of
// diffusion_radius, and the fourth-order Cahn-Hilliard operator M_c kappa
// lap^2 down to -M_c kappa (lx + ly)^2.  The limits:
//   heat       D = largest lambda / (rho C_p) of the phases (Eq. 4), odd walls
//              where the temperature is held;
//   momentum   D = 2 mu / rho (largest of the phases) + c_s^2 delta_t, the
//              compressive viscous mode of the flux (its face state adds
//              c_s^2 delta_t), odd walls except outlets;
//   phase      M_c (kappa l^2 + 2 beta l), l = lx + ly with mirrored walls,
//              2 beta the largest curvature of the double well (Sec. 2.3.1);
//   acoustic   c_s dt (1/wx + 1/wy) <= sqrt(3), wx, wy the smallest widths.
// Returns the first limit exceeded as text ("" if none).
std::string step_limits(const eulbfs_params* p)
{
    const bool px = p->bc[0].periodic != 0, py = p->bc[2].periodic != 0;
    auto radius = [&](bool xdir, auto odd) {
        const int s0 = xdir ? 0 : 2;
        return xdir ? diffusion_radius(p->x_width, p->dx, p->nx, px, odd(p->bc[s0]), odd(p->bc[s0 + 1]))
                    : diffusion_radius(p->y_width, p->dx, p->ny, py, odd(p->bc[s0]), odd(p->bc[s0 + 1]));
    };
    auto held_T = [](const eulbfs_bc& b) { return b.heat == EULBFS_HEAT_DIRICHLET; };
    auto held_M = [](const eulbfs_bc& b) { return b.flow != EULBFS_FLOW_OUTLET; };
    auto mirror = [](const eulbfs_bc&) { return false; };
    const double l_heat = radius(true, held_T) + radius(false, held_T);
    const double l_mom = radius(true, held_M) + radius(false, held_M);
    const double l_ch = radius(true, mirror) + radius(false, mirror);
    double d_heat = 0.0, nu = 0.0;
    for (int k = 0; k < 3; ++k) {
        d_heat = std::max(d_heat, p->lambda[k] / (p->rho[k] * p->cp[k]));
        nu = std::max(nu, p->mu[k] / p->rho[k]);
    }
    const double d_mom = 2.0 * nu + p->delta_t / 3.0;
    const double beta = 12.0 * p->sigma / p->xi, kappa = 1.5 * p->xi * p->sigma;
    const double wx = min_width(p->x_width, p->dx, p->nx), wy = min_width(p->y_width, p->dx, p->ny);
    const double re_bound = 2.51, im_bound = std::sqrt(3.0);
    const double v_heat = p->dt * d_heat * l_heat, v_mom = p->dt * d_mom * l_mom;
    const double v_ch = p->dt * p->mobility * (kappa * l_ch * l_ch + 2.0 * beta * l_ch);
    const double v_ac = p->dt * std::sqrt(1.0 / 3.0) * (1.0 / wx + 1.0 / wy);
    char buf[160];
    auto over = [&](const char* what, double v, double bound) {
        std::snprintf(buf, sizeof buf, "dt = %g is beyond the %s limit of the explicit RK3 step (%.4g > %.4g)",
                      p->dt, what, v, bound);
        return std::string(buf);
    };
    if (v_heat > re_bound) return over("thermal diffusion", v_heat, re_bound);
    if (v_mom > re_bound) return over("viscous", v_mom, re_bound);
    if (v_ch > re_bound) return over("Cahn-Hilliard", v_ch, re_bound);
    if (v_ac > im_bound) return over("acoustic", v_ac, im_bound);
    return "";
}

std::string check(const eulbfs_params* p)
{
    if (!p) return "params is NULL";
    if (p->struct_size != sizeof(eulbfs_params)) return "struct_size does not match sizeof(eulbfs_params)";
    if (p->abi_version != EULBFS_ABI_VERSION) return "abi_version mismatch";
    if (p->nx < 4 || p->ny < 4) return "nx and ny must be >= 4";
    if ((int64_t)p->nx * p->ny > (int64_t)1 << 31) return "grid too large";
    if (!(p->dx > 0)) return "dx must be > 0";
    const double wmin = std::min(min_width(p->x_width, p->dx, p->nx), min_width(p->y_width, p->dx, p->ny));
    if (!(wmin > 0)) return "cell widths must be finite and > 0";
    if (!(p->delta_t > 0) || p->delta_t > 0.5 * wmin * (1 + 1e-12))
        return "delta_t must satisfy 0 < delta_t <= half the smallest cell width (surrounding points inside the "
               "two cells)";
    if (!(p->dt > 0)) return "dt must be > 0";
    if (p->lattice_hg != 5 && p->lattice_hg != 9) return "lattice_hg must be 5 or 9";
    if (p->precision != EULBFS_FP64 && p->precision != EULBFS_FP32) return "unknown precision";
    if (p->kernel != EULBFS_KERNEL_FUSED && p->kernel != EULBFS_KERNEL_SPLIT && p->kernel != EULBFS_KERNEL_AUTO)
        return "unknown kernel variant";
    if (p->surf_model != 0 && p->surf_model != 1) return "surf_model must be 0 or 1";
    if (p->c_source != 0 && p->c_source != 1) return "c_source must be 0 or 1";
    for (int k = 0; k < 3; ++k) {
        if (!(p->rho[k] > 0)) return "densities must be > 0";
        if (!(p->mu[k] >= 0) || !(p->lambda[k] >= 0)) return "viscosities and conductivities must be >= 0";
        if (!(p->cp[k] > 0)) return "heat capacities must be > 0";
    }
    if (!(p->latent >= 0)) return "latent heat must be >= 0";
    if (!(p->T_l >= p->T_s)) return "T_l must be >= T_s";
    if (!(p->sigma >= 0)) return "sigma must be >= 0";
    if (!(p->xi > 0)) return "xi must be > 0";
    if (!(p->mobility >= 0) || !(p->Qg > 0)) return "mobility must be >= 0 and Qg > 0";
    if (!(p->xi >= 2.0 * wmin)) return "xi must span at least two cells (2 dx; the smallest width on a stretched mesh)";
    for (int a = 0; a < 2; ++a) {
        const eulbfs_bc& lo = p->bc[2 * a];
        const eulbfs_bc& hi = p->bc[2 * a + 1];
        if ((lo.periodic != 0) != (hi.periodic != 0)) return "periodic must agree on opposite sides";
    }
    for (int s = 0; s < 4; ++s) {
        const eulbfs_bc& b = p->bc[s];
        if (b.periodic) continue;
        if (b.flow < 0 || b.flow > 2) return "unknown flow boundary rule";
        if (b.heat < 0 || b.heat > 1) return "unknown heat boundary rule";
        if (!(b.theta_deg > 0 && b.theta_deg < 180)) return "contact angle must be in (0, 180) deg";
        if (b.theta_adv != 0.0 || b.theta_rec != 0.0) {
            if (!(b.theta_rec > 0 && b.theta_rec <= b.theta_deg && b.theta_deg <= b.theta_adv && b.theta_adv < 180))
                return "hysteresis window needs 0 < theta_rec <= theta_deg <= theta_adv < 180 deg";
        }
    }
    const int tiles[][2] = {{0, 0}, {32, 8}, {64, 4}, {16, 16}, {64, 8}, {32, 16}, {32, 32}};
    bool ok = false;
    for (auto& t : tiles) ok |= (p->tile_x == t[0] && p->tile_y == t[1]);
    if (!ok) return "tile must be 0x0, 32x8, 64x4, 16x16, 64x8, 32x16 or 32x32";
    return step_limits(p);
}

int tile_of(const eulbfs_params* p)
{
    if (p->tile_x == 64 && p->tile_y == 4) return TILE_64x4;
    if (p->tile_x == 16 && p->tile_y == 16) return TILE_16x16;
    if (p->tile_x == 64 && p->tile_y == 8) return TILE_64x8;
    if (p->tile_x == 32 && p->tile_y == 16) return TILE_32x16;
    if (p->tile_x == 32 && p->tile_y == 32) return TILE_32x32;
    return TILE_32x8;
}

DevParams make_dev(const eulbfs_params* p)
{
    DevParams d;
    std::memset(&d, 0, sizeof d);
    d.nx = p->nx;
    d.ny = p->ny;
    d.pitch = round_pitch(p->nx);
    d.lattice_hg = p->lattice_hg;
    d.surf_model = p->surf_model;
    d.c_source = p->c_source;
    d.periodic_x = p->bc[0].periodic ? 1 : 0;
    d.periodic_y = p->bc[2].periodic ? 1 : 0;
    for (int s = 0; s < 4; ++s) {
        d.flow[s] = p->bc[s].flow;
        d.heat[s] = p->bc[s].heat;
        d.T_w[s] = p->bc[s].T_w;
        d.wet[s] = p->dx * (4.0 / p->xi) * std::cos(p->bc[s].theta_deg * M_PI / 180.0);
        d.hyst[s] = (!p->bc[s].periodic && p->bc[s].theta_adv != 0.0) ? 1 : 0;
        d.cos_adv[s] = std::cos(p->bc[s].theta_adv * M_PI / 180.0);
        d.cos_rec[s] = std::cos(p->bc[s].theta_rec * M_PI / 180.0);
    }
    d.wet_k = p->dx * (4.0 / p->xi);
    d.dx = p->dx;
    d.inv_dx = 1.0 / p->dx;
    d.inv_2dx = 1.0 / (2.0 * p->dx);
    d.inv_dx2 = 1.0 / (p->dx * p->dx);
    d.delta_t = p->delta_t;
    d.dt = p->dt;
    d.inv_dt = 1.0 / p->dt;
    d.half_off[0] = 0.25;
    d.half_off[1] = 0.125;
    for (int k = 0; k < 3; ++k) {
        d.rho[k] = p->rho[k];
        d.mu[k] = p->mu[k];
        d.lam[k] = p->lambda[k];
        d.cp[k] = p->cp[k];
    }
    d.latent = p->latent;
    d.T_s = p->T_s;
    d.T_l = p->T_l;
    d.beta = 12.0 * p->sigma / p->xi;
    d.kappa = 1.5 * p->xi * p->sigma;
    d.a_g = p->mobility / (p->Qg * p->delta_t);
    d.muQ = p->Qg;
    d.cpref = 0.5 * (p->cp[0] + p->cp[1]);
    d.k_h = 3.0 / (d.cpref * p->delta_t);
    d.k_f = 3.0 / p->delta_t;
    d.gx = p->gx;
    d.gy = p->gy;
    d.expansion = 1.0 - p->rho[0] / p->rho[1];
    // compile-time fast paths valid for these constants (same quantities up to rounding)
    d.fast = (0.5 * p->dx - p->delta_t == 0.0 && !stretched(p) ? FAST_HALF : 0) |
             (p->cp[0] == p->cp[1] && p->cp[1] == p->cp[2] ? FAST_UCP : 0);
    d.Hs_u = p->cp[0] * p->T_s;
    d.Hl_u = p->cp[0] * p->T_l + p->latent;
    d.inv_cp = 1.0 / p->cp[0];
    d.inv_dH = d.Hl_u - d.Hs_u > 1e-300 ? 1.0 / (d.Hl_u - d.Hs_u) : 0.0;
    return d;
}

// Byte offsets of every region of a solver's workspace.
struct Layout {
    size_t mesh;         // stretched-mesh tables (mesh_bytes; 0 on a uniform mesh)
    size_t mesh_bytes;
    int msx, msy;        // ghosted columns / rows per table, padded
    size_t state_bytes;  // one copy of W
    size_t plane_R, plane_H;
    size_t W0, fsdot, WA, WB, staging, staging_bytes, red_partial, red_out;
    int red_blocks;
    bool split;
    size_t g, prim, Fx, Fy;  // split scratch
    int gpitch, fpitch;
    size_t gplane_H, gplane_R, pstride, fstride;
    size_t total;
};

Layout make_layout(const eulbfs_params* p)
{
    Layout L{};
    const size_t rs = p->precision == EULBFS_FP32 ? 4 : 8;
    const int pitch = round_pitch(p->nx);
    L.plane_H = align_up((size_t)p->ny * pitch * 8);
    L.plane_R = align_up((size_t)p->ny * pitch * rs);
    L.state_bytes = 2 * L.plane_H + 3 * L.plane_R;  // H and C in double, p and M in the field type
    size_t off = 0;
    L.W0 = off;
    off += L.state_bytes;
    L.fsdot = off;
    off += L.plane_R;
    // WA and WB are dead between steps: the same bytes stage dense double
    // planes for initialisation, checkpoints and queries.
    const size_t gn = (size_t)(p->nx + 2 * NG) * (p->ny + 2 * NG);
    L.staging_bytes = align_up(std::max((size_t)6 * p->nx * p->ny, 5 * gn) * 8);
    L.staging = off;
    L.WA = off;
    L.WB = off + L.state_bytes;
    off += std::max(2 * L.state_bytes, L.staging_bytes);
    const size_t ncell = (size_t)p->nx * p->ny;
    L.red_blocks = (int)std::min<size_t>(1024, (ncell + 255) / 256);
    L.red_partial = off;
    off += align_up((size_t)L.red_blocks * NRED * 8);
    L.red_out = off;
    off += align_up(16 * 8);
    L.split = p->kernel == EULBFS_KERNEL_SPLIT;
    L.gpitch = round_pitch(p->nx + 2 * NG);
    L.fpitch = round_pitch(p->nx + 1);
    L.gplane_H = align_up((size_t)(p->ny + 2 * NG) * L.gpitch * 8);  // H and C planes
    L.gplane_R = align_up((size_t)(p->ny + 2 * NG) * L.gpitch * rs);
    L.pstride = L.gplane_R / rs;
    L.fstride = align_up((size_t)(p->ny + 1) * L.fpitch * rs) / rs;
    if (L.split) {
        L.g = off;
        off += 2 * L.gplane_H + 3 * L.gplane_R;
        L.prim = off;
        off += (NPRIM + 1) * L.gplane_R;
        L.Fx = off;
        off += 5 * L.fstride * rs;
        L.Fy = off;
        off += 5 * L.fstride * rs;
    }
    if (stretched(p)) {
        L.msx = (p->nx + 2 * NG + 31) / 32 * 32;
        L.msy = (p->ny + 2 * NG + 31) / 32 * 32;
        L.mesh_bytes = align_up(((size_t)4 * MS_STRIDE + (size_t)NMESH * (L.msx + L.msy)) * 8);
        L.mesh = off;
        off += L.mesh_bytes;
    }
    L.total = off;
    return L;
}

// Geometry tables of a stretched mesh (layout of MESH_* and MS_* in the
// device header): mside[4][MS_STRIDE], then NMESH arrays of L.msx doubles
// over the ghosted columns, then NMESH arrays of L.msy over the ghosted rows.
// Ghost cells take the width of the cell they copy (the periodic image, or
// the interior cell k-1 that ghost layer k mirrors), so a wall lies midway
// between a ghost and its mirror.
std::vector<double> mesh_tables(const eulbfs_params* p, const Layout& L)
{
    std::vector<double> t((size_t)4 * MS_STRIDE + (size_t)NMESH * (L.msx + L.msy), 0.0);
    auto ghosted = [&](const double* w, int n, bool periodic) {
        std::vector<double> g(n + 2 * NG);
        for (int l = 0; l < n + 2 * NG; ++l) {
            const int i = l - NG;
            int src = i;
            if (i < 0 || i >= n) src = periodic ? (i % n + n) % n : (i < 0 ? -i - 1 : 2 * n - 1 - i);
            g[l] = w ? w[src] : p->dx;
        }
        return g;
    };
    auto fill = [&](const std::vector<double>& g, double* m, int stride) {
        const int gn = (int)g.size();
        for (int l = 0; l < gn; ++l) {
            m[MESH_HW * stride + l] = 0.5 * g[l];
            m[MESH_IW * stride + l] = 1.0 / g[l];
            if (l == 0 || l == gn - 1) continue;
            const double hm = 0.5 * (g[l - 1] + g[l]), hp = 0.5 * (g[l] + g[l + 1]), hs = hm + hp;
            // parabola through the centres at -hm, 0, +hp
            m[MESH_GM * stride + l] = -hp / (hm * hs);
            m[MESH_G0 * stride + l] = (hp - hm) / (hm * hp);
            m[MESH_GP * stride + l] = hm / (hp * hs);
            m[MESH_LM * stride + l] = 2.0 / (hm * hs);
            m[MESH_LP * stride + l] = 2.0 / (hp * hs);
            m[MESH_L0 * stride + l] = -(m[MESH_LM * stride + l] + m[MESH_LP * stride + l]);
        }
    };
    const std::vector<double> gx = ghosted(p->x_width, p->nx, p->bc[0].periodic != 0);
    const std::vector<double> gy = ghosted(p->y_width, p->ny, p->bc[2].periodic != 0);
    double* mx = t.data() + 4 * MS_STRIDE;
    double* my = mx + (size_t)NMESH * L.msx;
    fill(gx, mx, L.msx);
    fill(gy, my, L.msy);
    for (int sd = 0; sd < 4; ++sd) {
        const eulbfs_bc& b = p->bc[sd];
        double* ms = t.data() + sd * MS_STRIDE;
        if (b.periodic) continue;
        // centres of the first three interior cells, measured from the wall
        const std::vector<double>& g = sd < 2 ? gx : gy;
        const int n = sd < 2 ? p->nx : p->ny;
        double s[3], acc = 0.0;
        for (int m = 0; m < 3; ++m) {
            const double w = g[NG + ((sd & 1) ? n - 1 - m : m)];
            s[m] = acc + 0.5 * w;
            acc += w;
        }
        for (int k = 0; k < 3; ++k) ms[MS_D + k] = 2.0 * s[k];
        // d/ds at s = 0 of the Lagrange parabola through the three centres
        ms[MS_L0 + 0] = -(s[1] + s[2]) / ((s[0] - s[1]) * (s[0] - s[2]));
        ms[MS_L0 + 1] = -(s[0] + s[2]) / ((s[1] - s[0]) * (s[1] - s[2]));
        ms[MS_L0 + 2] = -(s[0] + s[1]) / ((s[2] - s[0]) * (s[2] - s[1]));
        ms[MS_K] = 4.0 / p->xi;
        ms[MS_WET] = ms[MS_K] * std::cos(b.theta_deg * M_PI / 180.0);
    }
    return t;
}

size_t split_scratch_bytes(const Layout& L, size_t rs)
{
    return 2 * L.gplane_H + 3 * L.gplane_R + (NPRIM + 1) * L.gplane_R + 10 * L.fstride * rs;
}

template <typename R>
State<R> state_at(char* base, size_t off, const Layout& L)
{
    State<R> s;
    s.H = (double*)(base + off);
    s.p = (R*)(base + off + L.plane_H);
    s.mx = (R*)(base + off + L.plane_H + L.plane_R);
    s.my = (R*)(base + off + L.plane_H + 2 * L.plane_R);
    s.C = (double*)(base + off + L.plane_H + 3 * L.plane_R);
    return s;
}

template <typename R>
SplitScratch<R> split_at(char* base, const Layout& L)
{
    SplitScratch<R> X;
    X.g.H = (double*)(base + L.g);
    X.g.p = (R*)(base + L.g + L.gplane_H);
    X.g.mx = (R*)(base + L.g + L.gplane_H + L.gplane_R);
    X.g.my = (R*)(base + L.g + L.gplane_H + 2 * L.gplane_R);
    X.g.C = (double*)(base + L.g + L.gplane_H + 3 * L.gplane_R);
    X.gpitch = L.gpitch;
    X.prim = (R*)(base + L.prim);
    X.pstride = L.pstride;
    X.Fx = (R*)(base + L.Fx);
    X.Fy = (R*)(base + L.Fy);
    X.fpitch = L.fpitch;
    X.fstride = L.fstride;
    return X;
}

template <typename R>
__global__ void k_to_double(const R* src, size_t spitch, int w, int h, double* dst)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i < w && j < h) dst[(size_t)j * w + i] = (double)src[(size_t)j * spitch + i];
}

template <typename R>
hipError_t to_double(const R* src, size_t spitch, int w, int h, double* dst, hipStream_t st)
{
    const dim3 b(64, 4), g((w + 63) / 64, (h + 3) / 4);
    hipLaunchKernelGGL(k_to_double<R>, g, b, 0, st, src, spitch, w, h, dst);
    return hipGetLastError();
}

}  // namespace

// Steps per captured graph of a single solver.
constexpr int GRAPH_STEPS = 8;
// Ticks a batch enqueues ahead of the device before eulbfs_batch_tick waits.
constexpr int MAX_INFLIGHT = 2;

struct eulbfs_solver {
    eulbfs_params prm;
    DevParams dp;
    Layout L;
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    bool own_ws = false;
    int tile = TILE_32x8;
    int sched = EULBFS_KERNEL_FUSED;  // FUSED or SPLIT (AUTO resolves to FUSED with a tuned tile)
    int64_t steps = 0;
    bool poisoned = false;
    std::string err;
    // GRAPH_STEPS steps captured once and replayed (kernel nodes only)
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    bool graph_failed = false;
    int device = -1;  // device current at create
};

namespace {

template <typename R>
int enqueue_raw(eulbfs_solver* h, int64_t n)
{
    std::string* err = &h->err;
    const DevParams& P = h->dp;
    const Layout& L = h->L;
    State<R> W0 = state_at<R>(h->ws, L.W0, L), WA = state_at<R>(h->ws, L.WA, L), WB = state_at<R>(h->ws, L.WB, L);
    R* fsdot = (R*)(h->ws + L.fsdot);
    const StageCoef K1{0.0, 1.0, 1.0, 0}, K2{0.75, 0.25, 0.25, 0}, K3{1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0, 1};
    for (int64_t s = 0; s < n; ++s) {
        if (h->sched == EULBFS_KERNEL_SPLIT) {
            const SplitScratch<R> X = split_at<R>(h->ws, L);
            HIP_TRY(launch_stage_split<R>(P, X, K1, W0, W0, WA, fsdot, nullptr, 0, h->stream));
            HIP_TRY(launch_stage_split<R>(P, X, K2, WA, W0, WB, fsdot, nullptr, 0, h->stream));
            HIP_TRY(launch_stage_split<R>(P, X, K3, WB, W0, W0, fsdot, nullptr, 0, h->stream));
        } else {
            HIP_TRY(launch_stage_fused<R>(P, h->tile, K1, W0, W0, WA, fsdot, h->stream));
            HIP_TRY(launch_stage_fused<R>(P, h->tile, K2, WA, W0, WB, fsdot, h->stream));
            HIP_TRY(launch_stage_fused<R>(P, h->tile, K3, WB, W0, W0, fsdot, h->stream));
        }
    }
    return EULBFS_OK;
}

// Capture GRAPH_STEPS steps into a graph (once per solver).  Capture needs a
// created stream; on the legacy default stream, or if capture fails, the
// solver keeps launching eagerly.
template <typename R>
bool ensure_graph(eulbfs_solver* h)
{
    if (h->graph_exec) return true;
    if (h->graph_failed || h->stream == nullptr) return false;
    if (hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        h->graph_failed = true;
        (void)hipGetLastError();
        return false;
    }
    const int rc = enqueue_raw<R>(h, GRAPH_STEPS);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(h->stream, &g);
    if (rc != EULBFS_OK || e != hipSuccess || !g ||
        hipGraphInstantiate(&h->graph_exec, g, nullptr, nullptr, 0) != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        h->graph_exec = nullptr;
        h->graph_failed = true;
        (void)hipGetLastError();
        return false;
    }
    h->graph = g;
    return true;
}

template <typename R>
int enqueue_steps(eulbfs_solver* h, int64_t n)
{
    std::string* err = &h->err;
    int64_t left = n;
    // the graph is captured at the first call (capture launches nothing), so
    // later calls, timed ones included, find it ready
    if (ensure_graph<R>(h)) {
        for (; left >= GRAPH_STEPS; left -= GRAPH_STEPS) HIP_TRY(hipGraphLaunch(h->graph_exec, h->stream));
    }
    const int rc = enqueue_raw<R>(h, left);
    if (rc != EULBFS_OK) return rc;
    h->steps += n;
    return EULBFS_OK;
}

// What is wrong with an initial-state description, or "".
std::string init_error(const eulbfs_init* init)
{
    if (!init) return "init is NULL";
    if (init->kind == EULBFS_INIT_ANALYTIC) {
        const eulbfs_shape* e = init->shape;
        if (!e) return "init->shape is NULL";
        if (e->profile < EULBFS_PROFILE_UNIFORM || e->profile > EULBFS_PROFILE_DROPLET) return "unknown shape profile";
        if (e->profile == EULBFS_PROFILE_LAYER && e->axis != 0 && e->axis != 1) return "layer axis must be 0 or 1";
        const double v[] = {e->c0, e->h0, e->x0, e->y0, e->r0, e->t_out, e->t_in, e->t_amp, e->fl0, e->u_in, e->v_in};
        for (double x : v)
            if (!std::isfinite(x)) return "shape values must be finite";
        if (e->fl0 < 0.0 || e->fl0 > 1.0) return "shape fl0 must be in [0, 1]";
        return "";
    }
    if (init->kind != EULBFS_INIT_PRIMITIVE && init->kind != EULBFS_INIT_CONSERVED) return "unknown init kind";
    if (!init->planes) return "init->planes is NULL";
    return "";
}

// Initial state from six planes or a closed-form shape.  With sync = false
// nothing waits: host planes must stay valid until the stream has run the
// copy (batch admission passes planes already on the device); a shape is
// read before the call returns.
template <typename R>
int do_init(eulbfs_solver* h, const eulbfs_init* init, bool sync = true)
{
    std::string* err = &h->err;
    const Layout& L = h->L;
    const size_t n6 = (size_t)6 * h->prm.nx * h->prm.ny;
    double* stage = (double*)(h->ws + L.staging);
    const double* src = init->planes;
    if (init->kind == EULBFS_INIT_ANALYTIC) {
        const eulbfs_shape& e = *init->shape;
        const InitShape S{e.profile, e.axis, e.c0,    e.h0,   e.x0, e.y0, e.r0, e.t_out,
                          e.t_in,    e.t_amp, e.seed, e.fl0, e.u_in, e.v_in, h->prm.xi};
        HIP_TRY(launch_init_shape(h->dp, S, stage, h->stream));
        src = stage;
    } else if (!init->on_device) {
        HIP_TRY(hipMemcpyAsync(stage, init->planes, n6 * 8, hipMemcpyHostToDevice, h->stream));
        src = stage;
    }
    State<R> W0 = state_at<R>(h->ws, L.W0, L);
    R* fsdot = (R*)(h->ws + L.fsdot);
    if (init->kind != EULBFS_INIT_CONSERVED)
        HIP_TRY(launch_init<R>(h->dp, src, W0, fsdot, h->stream));
    else
        HIP_TRY(launch_set_conserved<R>(h->dp, src, W0, fsdot, -1, h->stream));
    if (sync) HIP_TRY(hipStreamSynchronize(h->stream));
    return EULBFS_OK;
}

// The EULBFS_SCALAR_DIAG record from the raw reduction sums.
void diag_from_sums(const eulbfs_solver* h, const double r[NRED], double* out)
{
    // a stretched mesh weights each cell inside the sums
    const bool nu = h->dp.mside != nullptr;
    const double dV = nu ? 1.0 : h->prm.dx * h->prm.dx;
    const double dl = nu ? 1.0 : h->prm.dx;
    out[0] = r[RED_RHO] * dV;
    out[1] = r[RED_C] * dV;
    out[2] = r[RED_H] * dV;
    out[3] = r[RED_FS] * dV;
    out[4] = r[RED_UMAX];
    out[5] = r[RED_NONFINITE];
    out[6] = r[RED_TIP] * dl;
    out[7] = (double)h->steps * h->prm.dt;
    out[8] = (double)h->steps;
    out[9] = h->prm.dt;
    out[10] = -r[RED_NEG_CMIN];
    out[11] = r[RED_CMAX];
    out[12] = r[RED_WALL] * dl;
    out[13] = r[RED_AXIS] * dl;
}

// Watchdog on a diagnostics record: "" when the state is usable, else why not.
// F_s = clamp(C) (1 - F_l) lies in [0, 1] by construction, so the range check
// is on the order parameter it is built from.
std::string unstable_reason(const double d[EULBFS_NDIAG])
{
    if (d[5] != 0.0 || !std::isfinite(d[0]) || !std::isfinite(d[2]))
        return "non-finite values in the state";
    if (!(d[4] <= 1.0 / std::sqrt(3.0)))
        return "speed " + std::to_string(d[4]) + " above the lattice sound speed";
    if (!(d[10] >= -EULBFS_C_MARGIN && d[11] <= 1.0 + EULBFS_C_MARGIN))
        return "order parameter outside [" + std::to_string(-EULBFS_C_MARGIN) + ", " +
               std::to_string(1.0 + EULBFS_C_MARGIN) + "] (min " + std::to_string(d[10]) + ", max " +
               std::to_string(d[11]) + ")";
    return "";
}

template <typename R>
int do_diag(eulbfs_solver* h, double* host_out)
{
    std::string* err = &h->err;
    const Layout& L = h->L;
    State<R> W0 = state_at<R>(h->ws, L.W0, L);
    double* part = (double*)(h->ws + L.red_partial);
    double* dout = (double*)(h->ws + L.red_out);
    HIP_TRY(launch_reduce<R>(h->dp, W0, part, L.red_blocks, dout, h->stream));
    double r[NRED];
    HIP_TRY(hipMemcpyAsync(r, dout, sizeof r, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    diag_from_sums(h, r, host_out);
    return EULBFS_OK;
}

template <typename R>
int do_query_field(eulbfs_solver* h, int what, void* out, size_t bytes, int on_dev)
{
    std::string* err = &h->err;
    const Layout& L = h->L;
    const int nx = h->prm.nx, ny = h->prm.ny;
    const size_t n = (size_t)nx * ny;
    const size_t gn = (size_t)(nx + 2 * NG) * (ny + 2 * NG);
    size_t need = what == EULBFS_FIELD_W_ALL ? 6 * n * 8 : (what == EULBFS_FIELD_W_GHOSTED ? 5 * gn * 8 : n * 8);
    if (bytes < need) return set_err(err, EULBFS_EINVAL, "output buffer too small");
    State<R> W0 = state_at<R>(h->ws, L.W0, L);
    const R* fsdot = (const R*)(h->ws + L.fsdot);
    double* stage = (double*)(h->ws + L.staging);
    if (what == EULBFS_FIELD_W_ALL) {
        for (int k = 0; k < 6; ++k) HIP_TRY(launch_export<R>(h->dp, W0, fsdot, k, stage + k * n, h->stream));
    } else {
        HIP_TRY(launch_export<R>(h->dp, W0, fsdot, what, stage, h->stream));
    }
    HIP_TRY(hipMemcpyAsync(out, stage, need, on_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return EULBFS_OK;
}

template <typename R>
int do_set_field(eulbfs_solver* h, int what, const void* in, size_t bytes, int on_dev)
{
    std::string* err = &h->err;
    const Layout& L = h->L;
    const size_t n = (size_t)h->prm.nx * h->prm.ny;
    const size_t need = what == EULBFS_FIELD_W_ALL ? 6 * n * 8 : n * 8;
    if (bytes < need) return set_err(err, EULBFS_EINVAL, "input buffer too small");
    double* stage = (double*)(h->ws + L.staging);
    HIP_TRY(hipMemcpyAsync(stage, in, need, on_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, h->stream));
    State<R> W0 = state_at<R>(h->ws, L.W0, L);
    R* fsdot = (R*)(h->ws + L.fsdot);
    HIP_TRY(launch_set_conserved<R>(h->dp, stage, W0, fsdot, what == EULBFS_FIELD_W_ALL ? -1 : what, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    h->poisoned = false;
    return EULBFS_OK;
}

// Device scratch of one residual evaluation: the split scratch (unless the
// workspace holds one), the residual planes in the state's pitch layout and a
// dense double staging area for the copies out.
template <typename R>
size_t residual_scratch_bytes(const eulbfs_solver* h)
{
    const Layout& L = h->L;
    const size_t sb = L.split ? 0 : align_up(split_scratch_bytes(L, sizeof(R)));
    return sb + 5 * L.plane_R + align_up((size_t)5 * (h->prm.nx + 1) * (h->prm.ny + 1) * 8);
}

// ext: caller-provided scratch of residual_scratch_bytes<R>(h) bytes, or NULL
// to allocate it here (and free it before returning).
template <typename R>
int do_residual(eulbfs_solver* h, double* Rout, double* Fx, double* Fy, int on_dev, char* ext)
{
    std::string* err = &h->err;
    const Layout& L = h->L;
    const int nx = h->prm.nx, ny = h->prm.ny;
    const size_t rs = sizeof(R);
    const size_t sb = L.split ? 0 : align_up(split_scratch_bytes(L, rs));
    const size_t rbytes = 5 * L.plane_R;
    char* tmp = ext;
    if (!ext) HIP_TRY(hipMalloc(&tmp, residual_scratch_bytes<R>(h)));
    SplitScratch<R> X;
    if (L.split) {
        X = split_at<R>(h->ws, L);
    } else {
        Layout L2 = L;
        L2.g = 0;
        L2.prim = L2.g + 2 * L.gplane_H + 3 * L.gplane_R;
        L2.Fx = L2.prim + (NPRIM + 1) * L.gplane_R;
        L2.Fy = L2.Fx + 5 * L.fstride * rs;
        X = split_at<R>(tmp, L2);
    }
    R* res = (R*)(tmp + sb);
    double* dd = (double*)(tmp + sb + rbytes);
    State<R> W0 = state_at<R>(h->ws, L.W0, L);
    R* fsdot = (R*)(h->ws + L.fsdot);
    const StageCoef K{0.0, 1.0, 1.0, 0};
    const hipMemcpyKind kind = on_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    const size_t rstride = L.plane_R / rs;
    hipError_t e = launch_stage_split<R>(h->dp, X, K, W0, W0, W0, fsdot, res, rstride, h->stream);
    if (e == hipSuccess && Rout) {
        for (int k = 0; k < 5 && e == hipSuccess; ++k)
            e = to_double<R>(res + k * rstride, h->dp.pitch, nx, ny, dd + (size_t)k * nx * ny, h->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(Rout, dd, (size_t)5 * nx * ny * 8, kind, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    }
    if (e == hipSuccess && Fx) {
        for (int k = 0; k < 5 && e == hipSuccess; ++k)
            e = to_double<R>(X.Fx + k * X.fstride, X.fpitch, nx + 1, ny, dd + (size_t)k * (nx + 1) * ny, h->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(Fx, dd, (size_t)5 * (nx + 1) * ny * 8, kind, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    }
    if (e == hipSuccess && Fy) {
        for (int k = 0; k < 5 && e == hipSuccess; ++k)
            e = to_double<R>(X.Fy + k * X.fstride, X.fpitch, nx, ny + 1, dd + (size_t)k * nx * (ny + 1), h->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(Fy, dd, (size_t)5 * nx * (ny + 1) * 8, kind, h->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (!ext) {
        const hipError_t ef = hipFree(tmp);
        if (e == hipSuccess) e = ef;
    }
    if (e != hipSuccess) return set_err(err, EULBFS_EDEVICE, std::string("residual: ") + hipGetErrorString(e));
    return EULBFS_OK;
}

// ---------------------------------------------------------------------------
// Tile autotuner.
//
// EULBFS_KERNEL_AUTO times the fused stage kernel with every tile shape for a
// few steps on the solver's own initial state, keeps the fastest and
// initialises the state again.  The tile shape does not change any cell's
// arithmetic, so the choice only changes the speed.  Choices are cached per
// process by grid size, precision, lattice, fast-path flags and periodicity.
// ---------------------------------------------------------------------------
struct TuneKey {
    int nx, ny, precision, lattice, fast, px, py;
    bool operator<(const TuneKey& o) const
    {
        return std::tie(nx, ny, precision, lattice, fast, px, py) <
               std::tie(o.nx, o.ny, o.precision, o.lattice, o.fast, o.px, o.py);
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune;  // -> tile

template <typename R>
int autotune(eulbfs_solver* h, const eulbfs_init* init)
{
    std::string* err = &h->err;
    const TuneKey key{h->prm.nx, h->prm.ny, h->prm.precision, h->prm.lattice_hg, h->dp.fast,
                      h->dp.periodic_x, h->dp.periodic_y};
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            h->tile = it->second;
            return EULBFS_OK;
        }
    }
    // about a millisecond of work per timing, at least two steps
    const double cells = (double)h->prm.nx * h->prm.ny;
    const int steps = (int)std::max(2.0, std::min(32.0, 4.0e6 / cells));
    hipEvent_t a = nullptr, b = nullptr;
    HIP_TRY(hipEventCreate(&a));
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return set_err(err, EULBFS_EDEVICE, "autotune: hipEventCreate failed");
    }
    // best of three per shape, the shapes taken in turn within each round so
    // that a drift of the clock during the trials weighs on all of them alike
    float ms[NTILES] = {};
    int rc = EULBFS_OK;
    for (int rep = 0; rep < 3 && rc == EULBFS_OK; ++rep) {
        for (int tile = 0; tile < NTILES && rc == EULBFS_OK; ++tile) {
            h->tile = tile;
            rc = enqueue_raw<R>(h, 1);
            float t = 0.0f;
            if (rc == EULBFS_OK &&
                (hipEventRecord(a, h->stream) != hipSuccess || enqueue_raw<R>(h, steps) != EULBFS_OK ||
                 hipEventRecord(b, h->stream) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
                 hipEventElapsedTime(&t, a, b) != hipSuccess))
                rc = set_err(err, EULBFS_EDEVICE, "autotune: a timed launch failed");
            if (rc == EULBFS_OK && (rep == 0 || t < ms[tile])) ms[tile] = t;
        }
    }
    int best = 0;
    for (int tile = 1; tile < NTILES; ++tile)
        if (ms[tile] < ms[best]) best = tile;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc != EULBFS_OK) return rc;
    h->tile = best;
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tune[key] = best;
    }
    return do_init<R>(h, init);  // the timed steps advanced the state
}

template <typename R>
int setup_schedule(eulbfs_solver* h, const eulbfs_init* init)
{
    if (h->L.split) {
        h->sched = EULBFS_KERNEL_SPLIT;
        return EULBFS_OK;
    }
    h->sched = EULBFS_KERNEL_FUSED;
    if (h->dp.mside) {  // a stretched mesh has one fused tile shape per field type
        static_assert(NuTile<double>::TX == 32 && NuTile<double>::TY == 16 && NuTile<float>::TX == 32 &&
                          NuTile<float>::TY == 32,
                      "the stretched-mesh tiles are reported as TILE_32x16 (FP64) and TILE_32x32 (FP32)");
        h->tile = h->prm.precision == EULBFS_FP32 ? TILE_32x32 : TILE_32x16;
        return EULBFS_OK;
    }
    if (h->prm.kernel == EULBFS_KERNEL_AUTO) return autotune<R>(h, init);
    return EULBFS_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int eulbfs_check_params(const eulbfs_params* prm, char* msg, size_t msg_len)
{
    const std::string e = check(prm);
    if (msg && msg_len) {
        std::snprintf(msg, msg_len, "%s", e.c_str());
    }
    if (!e.empty()) return set_err(nullptr, EULBFS_EINVAL, e);
    return EULBFS_OK;
}

size_t eulbfs_workspace_bytes(const eulbfs_params* prm)
{
    if (!check(prm).empty()) return 0;
    return make_layout(prm).total;
}

}  // extern "C"

namespace {

void free_solver(eulbfs_solver* h, bool sync);

// eulbfs_create; with sync = false the initial state is only enqueued, and a
// stretched mesh's tables must already be on their way to the workspace (the
// batch stages them through pinned memory).
int create_solver(const eulbfs_params* prm, const eulbfs_init* init, void* d_ws, size_t ws_bytes, void* hip_stream,
                  bool sync, eulbfs_solver** out)
{
    std::string* err = nullptr;
    if (!out) return set_err(err, EULBFS_EINVAL, "out is NULL");
    *out = nullptr;
    const std::string e = check(prm);
    if (!e.empty()) return set_err(err, EULBFS_EINVAL, e);
    const std::string ie = init_error(init);
    if (!ie.empty()) return set_err(err, EULBFS_EINVAL, ie);
    const Layout L = make_layout(prm);
    if (d_ws && ws_bytes < L.total) return set_err(err, EULBFS_ENOMEM, "workspace smaller than eulbfs_workspace_bytes()");
    if (d_ws && ((uintptr_t)d_ws % ALIGN) != 0) return set_err(err, EULBFS_EINVAL, "workspace must be 256-byte aligned");
    eulbfs_solver* h = new eulbfs_solver();
    h->prm = *prm;
    h->prm.x_width = nullptr;  // the caller's arrays live on in the mesh tables only
    h->prm.y_width = nullptr;
    h->dp = make_dev(prm);
    h->L = L;
    h->stream = (hipStream_t)hip_stream;
    h->tile = tile_of(prm);
    if (hipGetDevice(&h->device) != hipSuccess) h->device = -1;
    if (d_ws) {
        h->ws = (char*)d_ws;
    } else {
        hipError_t he = hipMalloc(&h->ws, L.total);
        if (he != hipSuccess) {
            delete h;
            return set_err(err, EULBFS_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(he));
        }
        h->own_ws = true;
    }
    if (L.mesh_bytes) {
        if (sync) {
            const std::vector<double> t = mesh_tables(prm, L);
            hipError_t he = hipMemcpy(h->ws + L.mesh, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice);
            if (he != hipSuccess) {
                free_solver(h, false);
                return set_err(err, EULBFS_EDEVICE, std::string("hipMemcpy (mesh tables): ") + hipGetErrorString(he));
            }
        }
        const double* base = (const double*)(h->ws + L.mesh);
        h->dp.mside = base;
        h->dp.mxc = base + 4 * MS_STRIDE;
        h->dp.myc = h->dp.mxc + (size_t)NMESH * L.msx;
        h->dp.msx = L.msx;
        h->dp.msy = L.msy;
    }
    int rc = prm->precision == EULBFS_FP32 ? do_init<float>(h, init, sync) : do_init<double>(h, init, sync);
    if (rc == EULBFS_OK)
        rc = prm->precision == EULBFS_FP32 ? setup_schedule<float>(h, init) : setup_schedule<double>(h, init);
    if (rc != EULBFS_OK) {
        g_thread_err = h->err;
        eulbfs_destroy(h);
        return rc;
    }
    *out = h;
    return EULBFS_OK;
}

// Release a solver's host state; sync = false when no enqueued work can
// still touch its workspace.
void free_solver(eulbfs_solver* h, bool sync)
{
    if (sync && (h->stream || h->ws)) (void)hipStreamSynchronize(h->stream);
    if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    if (h->own_ws && h->ws) (void)hipFree(h->ws);
    delete h;
}

}  // namespace

extern "C" {

int eulbfs_create(const eulbfs_params* prm, const eulbfs_init* init, void* d_ws, size_t ws_bytes, void* hip_stream,
                  eulbfs_solver** out)
{
    return create_solver(prm, init, d_ws, ws_bytes, hip_stream, true, out);
}

int eulbfs_step(eulbfs_t h, int64_t nsteps)
{
    if (!h) return set_err(nullptr, EULBFS_EINVAL, "handle is NULL");
    if (nsteps < 0) return set_err(&h->err, EULBFS_EINVAL, "nsteps must be >= 0");
    if (h->poisoned) return set_err(&h->err, EULBFS_EUNSTABLE, "state is unstable (non-finite or supersonic); restore a checkpoint");
    return h->prm.precision == EULBFS_FP32 ? enqueue_steps<float>(h, nsteps) : enqueue_steps<double>(h, nsteps);
}

int eulbfs_run(eulbfs_t h, int64_t nsteps, double t_end)
{
    if (!h) return set_err(nullptr, EULBFS_EINVAL, "handle is NULL");
    if (nsteps < 0) return set_err(&h->err, EULBFS_EINVAL, "nsteps must be >= 0");
    if (std::isnan(t_end)) return set_err(&h->err, EULBFS_EINVAL, "t_end is NaN");
    // the fixed step reaches t_end after ceil((t_end - t) / dt) more steps
    // (to a relative 1e-12, so that t_end = t + k dt takes exactly k steps)
    const double t = (double)h->steps * h->prm.dt;
    if (t_end < INFINITY) {
        const double k = std::ceil((t_end - t) / h->prm.dt * (1.0 - 1e-12));
        nsteps = std::min(nsteps, (int64_t)std::max(0.0, std::min(k, 9.0e18)));
    }
    int rc = eulbfs_step(h, nsteps);
    if (rc != EULBFS_OK) return rc;
    double d[EULBFS_NDIAG];
    rc = h->prm.precision == EULBFS_FP32 ? do_diag<float>(h, d) : do_diag<double>(h, d);
    if (rc != EULBFS_OK) return rc;
    const std::string why = unstable_reason(d);
    if (!why.empty()) {
        h->poisoned = true;
        return set_err(&h->err, EULBFS_EUNSTABLE, why + " after step " + std::to_string(h->steps));
    }
    return EULBFS_OK;
}

int eulbfs_query(eulbfs_t h, int32_t what, void* out, size_t bytes, int32_t out_on_device)
{
    if (!h) return set_err(nullptr, EULBFS_EINVAL, "handle is NULL");
    if (!out) return set_err(&h->err, EULBFS_EINVAL, "out is NULL");
    if (what == EULBFS_SCALAR_DIAG) {
        if (bytes < EULBFS_NDIAG * sizeof(double)) return set_err(&h->err, EULBFS_EINVAL, "output buffer too small");
        double d[EULBFS_NDIAG];
        int rc = h->prm.precision == EULBFS_FP32 ? do_diag<float>(h, d) : do_diag<double>(h, d);
        if (rc != EULBFS_OK) return rc;
        if (out_on_device) {
            hipError_t e = hipMemcpy(out, d, sizeof d, hipMemcpyHostToDevice);
            if (e != hipSuccess) return set_err(&h->err, EULBFS_EDEVICE, hipGetErrorString(e));
        } else {
            std::memcpy(out, d, sizeof d);
        }
        const std::string why = unstable_reason(d);
        if (!why.empty()) {
            h->poisoned = true;
            return set_err(&h->err, EULBFS_EUNSTABLE, why + " at step " + std::to_string(h->steps));
        }
        if (h->poisoned) return set_err(&h->err, EULBFS_EUNSTABLE, "state is unstable; restore a checkpoint");
        return EULBFS_OK;
    }
    if (what < 0 || what > EULBFS_FIELD_W_GHOSTED) return set_err(&h->err, EULBFS_EINVAL, "unknown selector");
    const int rc = h->prm.precision == EULBFS_FP32 ? do_query_field<float>(h, what, out, bytes, out_on_device)
                                                   : do_query_field<double>(h, what, out, bytes, out_on_device);
    if (rc == EULBFS_OK && h->poisoned)
        return set_err(&h->err, EULBFS_EUNSTABLE, "state is unstable; restore a checkpoint");
    return rc;
}

int eulbfs_set_field(eulbfs_t h, int32_t what, const void* in, size_t bytes, int32_t in_on_device)
{
    if (!h) return set_err(nullptr, EULBFS_EINVAL, "handle is NULL");
    if (!in) return set_err(&h->err, EULBFS_EINVAL, "in is NULL");
    if (!(what >= EULBFS_FIELD_H && what <= EULBFS_FIELD_FSDOT) && what != EULBFS_FIELD_W_ALL)
        return set_err(&h->err, EULBFS_EINVAL, "only conserved planes, dF_s/dt or W_ALL can be set");
    return h->prm.precision == EULBFS_FP32 ? do_set_field<float>(h, what, in, bytes, in_on_device)
                                           : do_set_field<double>(h, what, in, bytes, in_on_device);
}

int eulbfs_residual(eulbfs_t h, double* R, double* Fx, double* Fy, int32_t on_device)
{
    if (!h) return set_err(nullptr, EULBFS_EINVAL, "handle is NULL");
    return h->prm.precision == EULBFS_FP32 ? do_residual<float>(h, R, Fx, Fy, on_device, nullptr)
                                           : do_residual<double>(h, R, Fx, Fy, on_device, nullptr);
}

int eulbfs_residual_noalloc(eulbfs_t h, double* R, double* Fx, double* Fy, int32_t on_device)
{
    if (!h) return set_err(nullptr, EULBFS_EINVAL, "handle is NULL");
    const size_t need = h->prm.precision == EULBFS_FP32 ? residual_scratch_bytes<float>(h)
                                                        : residual_scratch_bytes<double>(h);
    if (need > EULBFS_NOALLOC_SCRATCH_BYTES)
        return set_err(&h->err, EULBFS_EINVAL,
                       "residual_noalloc: the grid needs " + std::to_string(need) +
                           " bytes of scratch, more than the static " +
                           std::to_string((size_t)EULBFS_NOALLOC_SCRATCH_BYTES));
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != h->device)
        return set_err(&h->err, EULBFS_EINVAL, "residual_noalloc: the solver's device must be current");
    char* scr = nullptr;
    if (int rc = noalloc_scratch(dev, &scr, &h->err)) return rc;
    return h->prm.precision == EULBFS_FP32 ? do_residual<float>(h, R, Fx, Fy, on_device, scr)
                                           : do_residual<double>(h, R, Fx, Fy, on_device, scr);
}

int eulbfs_destroy(eulbfs_t h)
{
    if (h) free_solver(h, true);
    return EULBFS_OK;
}

int eulbfs_schedule(eulbfs_t h, int32_t* kernel, int32_t* tile_x, int32_t* tile_y)
{
    if (!h) return set_err(nullptr, EULBFS_EINVAL, "handle is NULL");
    static const int TX[NTILES] = {32, 64, 16, 64, 32, 32}, TY[NTILES] = {8, 4, 16, 8, 16, 32};
    const bool split = h->sched == EULBFS_KERNEL_SPLIT;
    if (kernel) *kernel = h->sched;
    if (tile_x) *tile_x = split ? 0 : TX[h->tile];
    if (tile_y) *tile_y = split ? 0 : TY[h->tile];
    return EULBFS_OK;
}

const char* eulbfs_last_error(eulbfs_t h)
{
    if (!h) return g_thread_err.c_str();
    return h->err.c_str();
}

}  // extern "C"

// ===========================================================================
// Batched solves
//
// A batch owns one arena of device memory.  Each admitted request becomes a
// solver whose workspace is a range of the arena, so initialisation, queries
// and checkpoints are the single-solver code.  A tick advances every resident
// unfinished request by the same number of steps with one launch per RK stage
// over the concatenated tile lists of all of them.
// ===========================================================================
namespace {

struct Slot {
    eulbfs_solver* s = nullptr;
    size_t off = 0, bytes = 0;
    int64_t nsteps = 0, done = 0;
    int64_t finish_tick = -1;  // tick whose launches complete the request
    int64_t serial = -1;       // admission number: names the request (and so its tiles) in a graph key
};

struct TickEvent {
    hipEvent_t ev = nullptr;
    int64_t tick = -1;
    // the tick's step launches, timed for the tile choice; sig names the work
    // (step count and requests), so two ticks of equal sig did the same work
    hipEvent_t t0 = nullptr, t1 = nullptr;
    int tile = 0;
    double cell_steps = 0.0;
    uint64_t sig = 0;
};

}  // namespace

struct eulbfs_batch {
    size_t budget = 0;
    int max_slots = 0;
    int precision = EULBFS_FP64;
    char* base = nullptr;  // whole allocation: tables, then the arena
    bool own = false;
    hipStream_t stream = nullptr;
    char* arena = nullptr;
    size_t arena_bytes = 0;
    std::vector<Slot> slots;
    std::vector<std::pair<size_t, size_t>> free_list;  // (offset, bytes), sorted by offset
    // device tables (two sets, alternating between ticks)
    char* d_desc[2] = {nullptr, nullptr};
    int* d_tiles[2] = {nullptr, nullptr};
    size_t desc_bytes = 0;
    int tile_cap = 0;
    // pinned host copies of the tables
    char* h_desc[2] = {nullptr, nullptr};
    int* h_tiles[2] = {nullptr, nullptr};
    hipEvent_t upload_done[2] = {nullptr, nullptr};
    // per table set: a tick's launches (its steps x three stages x every group
    // present) captured for the step count and requests it was captured with
    // (their serials, in launch order), replayed while both are unchanged
    hipGraphExec_t step_graph[2] = {nullptr, nullptr};
    std::vector<int64_t> graph_key[2];
    std::vector<int64_t> last_key;  // requests of the previous tick
    bool graph_off = false;  // capture is impossible (legacy stream) or failed once
    // tile shape of uniform-mesh requests (EULBFS_BATCH_TILE_*) and what the
    // automatic choice has measured: device time and cell-steps of the timed
    // ticks of each shape; the running mean of log(t(64x8) / t(32x16)) over
    // back-to-back ticks of the same work; the last completed timed tick
    int tile_mode = EULBFS_BATCH_TILE_AUTO;
    double tile_ms[NBATCH_TILES] = {}, tile_cells[NBATCH_TILES] = {};
    int64_t tile_ticks[NBATCH_TILES] = {};
    double log_ratio = 0.0;
    int64_t pairs = 0;
    bool have_last = false;
    uint64_t last_sig = 0;
    int last_tile = 0;
    double last_ns = 0.0;
    int64_t admitted = 0;    // admissions so far
    int parity = 0;
    int64_t tick = 0;
    std::vector<TickEvent> events;  // recent ticks
    int64_t completed_tick = 0;     // every tick < completed_tick has completed
    // results and uploads that need no host wait: the reduction sums of each
    // request, copied into pinned memory by the tick that finishes it; host
    // initial planes staged in pinned memory and copied on an upload stream
    double* h_sums = nullptr;  // max_slots x NRED
    hipStream_t upload = nullptr;
    double* h_stage = nullptr;
    size_t stage_cap = 0;  // doubles
    hipEvent_t stage_done = nullptr;
    std::string err;
};

namespace {

size_t arena_alloc(eulbfs_batch* b, size_t bytes)
{
    for (size_t k = 0; k < b->free_list.size(); ++k) {
        auto& f = b->free_list[k];
        if (f.second >= bytes) {
            const size_t off = f.first;
            f.first += bytes;
            f.second -= bytes;
            if (f.second == 0) b->free_list.erase(b->free_list.begin() + k);
            return off;
        }
    }
    return SIZE_MAX;
}

void arena_free(eulbfs_batch* b, size_t off, size_t bytes)
{
    auto& fl = b->free_list;
    auto it = std::lower_bound(fl.begin(), fl.end(), std::make_pair(off, (size_t)0));
    it = fl.insert(it, {off, bytes});
    // merge with the next and the previous ranges
    if (it + 1 != fl.end() && it->first + it->second == (it + 1)->first) {
        it->second += (it + 1)->second;
        fl.erase(it + 1);
    }
    if (it != fl.begin() && (it - 1)->first + (it - 1)->second == it->first) {
        (it - 1)->second += it->second;
        fl.erase(it);
    }
}

eulbfs_params batch_view(const eulbfs_params* prm)
{
    eulbfs_params p = *prm;
    p.kernel = EULBFS_KERNEL_FUSED;  // batches step with the batched fused kernel
    p.tile_x = 0;
    p.tile_y = 0;
    return p;
}

size_t desc_size(int precision)
{
    return precision == EULBFS_FP32 ? sizeof(BatchDesc<float>) : sizeof(BatchDesc<double>);
}

// Mark ticks whose event has completed (non-blocking unless wait).
void batch_progress(eulbfs_batch* b, bool wait)
{
    while (!b->events.empty()) {
        TickEvent& te = b->events.front();
        const hipError_t e = wait ? hipEventSynchronize(te.ev) : hipEventQuery(te.ev);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            break;
        }
        b->completed_tick = te.tick + 1;
        float ms = 0.0f;
        if (te.t0 && te.t1 && te.cell_steps > 0.0 && hipEventElapsedTime(&ms, te.t0, te.t1) == hipSuccess) {
            const double ns = 1e6 * (double)ms / te.cell_steps;
            b->tile_ms[te.tile] += ms;
            b->tile_cells[te.tile] += te.cell_steps;
            ++b->tile_ticks[te.tile];
            if (b->have_last && b->last_sig == te.sig && b->last_tile != te.tile && b->last_ns > 0.0 && ns > 0.0) {
                const double r = te.tile == 1 ? std::log(ns / b->last_ns) : std::log(b->last_ns / ns);
                b->log_ratio = b->pairs == 0 ? r : b->log_ratio + 0.125 * (r - b->log_ratio);
                ++b->pairs;
            }
            b->have_last = true;
            b->last_sig = te.sig;
            b->last_tile = te.tile;
            b->last_ns = ns;
        } else {
            (void)hipGetLastError();
            b->have_last = false;
        }
        if (te.t0) (void)hipEventDestroy(te.t0);
        if (te.t1) (void)hipEventDestroy(te.t1);
        (void)hipEventDestroy(te.ev);
        b->events.erase(b->events.begin());
    }
}

// Tile shape of the next tick's uniform-mesh requests (an index into
// BATCH_TX/BATCH_TY): the pinned one; else, until a pair of back-to-back
// ticks of the same work has been timed on the two shapes, alternate; then
// the shape the paired ratios favour, with every EULBFS_BATCH_EXPLORE-th
// tick on the other.  The time of a tick depends on its requests far more
// than on its tile, so only ticks of the same work are compared; a mix that
// yields no pair within 32 ticks of each shape is judged by its summed
// times instead.
int batch_pick_tile(const eulbfs_batch* b)
{
    if (b->tile_mode != EULBFS_BATCH_TILE_AUTO) return b->tile_mode - 1;
    int best;
    if (b->pairs > 0) {
        best = b->log_ratio < 0.0 ? 1 : 0;
    } else if (b->tile_ticks[0] >= 4 * EULBFS_BATCH_EXPLORE && b->tile_ticks[1] >= 4 * EULBFS_BATCH_EXPLORE) {
        // a mix that never repeats a tick's work: fall back on the time per
        // cell-step summed over all timed ticks of each shape
        best = b->tile_ms[1] * b->tile_cells[0] < b->tile_ms[0] * b->tile_cells[1] ? 1 : 0;
    } else {
        return (int)(b->tick & 1);
    }
    return b->tick % EULBFS_BATCH_EXPLORE == EULBFS_BATCH_EXPLORE - 1 ? 1 - best : best;
}

template <typename R>
int batch_tick(eulbfs_batch* b, int32_t steps)
{
    std::string* err = &b->err;
    // active requests and the common step count of this tick
    std::vector<int> act;
    int64_t s_eff = steps;
    for (int k = 0; k < b->max_slots; ++k) {
        const Slot& sl = b->slots[k];
        if (sl.s && sl.done < sl.nsteps) {
            act.push_back(k);
            s_eff = std::min<int64_t>(s_eff, sl.nsteps - sl.done);
        }
    }
    if (act.empty() || s_eff <= 0) return EULBFS_OK;
    // at most MAX_INFLIGHT ticks enqueued ahead of the device
    while ((int)b->events.size() >= MAX_INFLIGHT) {
        const size_t before = b->events.size();
        batch_progress(b, true);
        if (b->events.size() == before) return set_err(err, EULBFS_EDEVICE, "waiting for a tick failed");
    }
    const int par = b->parity;
    b->parity ^= 1;
    if (b->upload_done[par]) HIP_TRY(hipEventSynchronize(b->upload_done[par]));
    BatchDesc<R>* hd = reinterpret_cast<BatchDesc<R>*>(b->h_desc[par]);
    int* ht = b->h_tiles[par];
    // tiles grouped by mesh kind, lattice and fast-path flags: one launch per
    // group present, each on its own sub-list of tiles, so a request's first
    // tile is counted from the start of its group
    constexpr int NGROUP = 16;
    auto group_of = [](const eulbfs_solver* h) {
        return (h->dp.mside ? 8 : 0) + (h->prm.lattice_hg == 5 ? 4 : 0) + (h->dp.fast & (FAST_HALF | FAST_UCP));
    };
    int ntiles[NGROUP] = {}, first[NGROUP] = {}, nd = 0;
    std::vector<int> order;
    for (int g = 0; g < NGROUP; ++g)
        for (int k : act)
            if (group_of(b->slots[k].s) == g) order.push_back(k);
    const int tile = batch_pick_tile(b);
    int tile_total = 0;
    double cells = 0.0;
    for (int k : order) {
        eulbfs_solver* h = b->slots[k].s;
        const int tb = h->dp.mside ? 0 : tile;  // stretched meshes: always the first shape
        const int tx = (h->prm.nx + BATCH_TX[tb] - 1) / BATCH_TX[tb];
        const int ty = (h->prm.ny + BATCH_TY[tb] - 1) / BATCH_TY[tb];
        cells += (double)h->prm.nx * h->prm.ny;
        if (tile_total + tx * ty > b->tile_cap) return set_err(err, EULBFS_ENOMEM, "batch tile table full");
        const int group = group_of(h);
        if (ntiles[group] == 0) first[group] = tile_total;
        BatchDesc<R>& D = hd[nd];
        D.P = h->dp;
        D.W[0] = state_at<R>(h->ws, h->L.W0, h->L);
        D.W[1] = state_at<R>(h->ws, h->L.WA, h->L);
        D.W[2] = state_at<R>(h->ws, h->L.WB, h->L);
        D.fsdot = (R*)(h->ws + h->L.fsdot);
        D.tiles_x = tx;
        D.tile0 = ntiles[group];
        for (int t = 0; t < tx * ty; ++t) ht[tile_total + t] = nd;
        tile_total += tx * ty;
        ntiles[group] += tx * ty;
        ++nd;
    }
    HIP_TRY(hipMemcpyAsync(b->d_desc[par], hd, (size_t)nd * sizeof(BatchDesc<R>), hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipMemcpyAsync(b->d_tiles[par], ht, (size_t)tile_total * sizeof(int), hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipEventRecord(b->upload_done[par], b->stream));
    const BatchDesc<R>* dd = reinterpret_cast<const BatchDesc<R>*>(b->d_desc[par]);
    const StageCoef K[3] = {{0.0, 1.0, 1.0, 0}, {0.75, 0.25, 0.25, 0}, {1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0, 1}};
    auto one_step = [&]() -> hipError_t {
        for (int stage = 0; stage < 3; ++stage)
            for (int g = 0; g < NGROUP; ++g)
                if (ntiles[g]) {
                    const hipError_t e = launch_stage_batched<R>(dd, b->d_tiles[par] + first[g], ntiles[g],
                                                                 (g & 4) ? 5 : 9, g & 3, g >= 8, g >= 8 ? 0 : tile,
                                                                 K[stage], stage, b->stream);
                    if (e != hipSuccess) return e;
                }
        return hipSuccess;
    };
    // The launches of a tick depend only on its step count, the requests
    // (their tables, tiles and groups) and the table set: a graph captured for
    // them is replayed; a new set is captured again (kernel nodes only).
    std::vector<int64_t> key{s_eff, tile};
    for (int k : order) key.push_back(b->slots[k].serial);
    uint64_t sig = 1469598103934665603ull;  // FNV-1a over the step count and the requests, not the tile
    for (size_t q = 0; q < key.size(); ++q)
        if (q != 1) sig = (sig ^ (uint64_t)key[q]) * 1099511628211ull;
    // a set of requests is captured once it has lasted a tick: in a busy
    // serving mix the set changes nearly every tick, and capturing each one
    // would cost more host time than the launches it replaces
    const bool steady = key == b->last_key;
    b->last_key = key;
    bool graph = false;
    if (!b->graph_off && b->stream != nullptr && s_eff > 1 && steady) {
        if (b->step_graph[par] && b->graph_key[par] == key) {
            graph = true;
        } else {
            if (b->step_graph[par]) (void)hipGraphExecDestroy(b->step_graph[par]);
            b->step_graph[par] = nullptr;
            hipGraph_t gr = nullptr;
            if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) == hipSuccess) {
                hipError_t el = hipSuccess;
                for (int64_t st = 0; st < s_eff && el == hipSuccess; ++st) el = one_step();
                const hipError_t ec = hipStreamEndCapture(b->stream, &gr);
                graph = el == hipSuccess && ec == hipSuccess && gr &&
                        hipGraphInstantiate(&b->step_graph[par], gr, nullptr, nullptr, 0) == hipSuccess;
            }
            if (gr) (void)hipGraphDestroy(gr);
            if (graph) {
                b->graph_key[par] = key;
            } else {  // launch eagerly from now on
                if (b->step_graph[par]) (void)hipGraphExecDestroy(b->step_graph[par]);
                b->step_graph[par] = nullptr;
                b->graph_off = true;
                (void)hipGetLastError();
            }
        }
    }
    TickEvent te;
    te.tile = tile;
    te.cell_steps = cells * (double)s_eff;
    te.sig = sig;
    if (hipEventCreate(&te.t0) != hipSuccess || hipEventCreate(&te.t1) != hipSuccess) {
        (void)hipGetLastError();  // untimed tick
        if (te.t0) (void)hipEventDestroy(te.t0);
        te.t0 = te.t1 = nullptr;
    }
    if (te.t0) HIP_TRY(hipEventRecord(te.t0, b->stream));
    if (graph)
        HIP_TRY(hipGraphLaunch(b->step_graph[par], b->stream));
    else
        for (int64_t st = 0; st < s_eff; ++st) HIP_TRY(one_step());
    if (te.t1) HIP_TRY(hipEventRecord(te.t1, b->stream));
    // requests finished by this tick: their FP64 sums go to pinned memory
    for (int k : act) {
        Slot& sl = b->slots[k];
        if (sl.done + s_eff < sl.nsteps) continue;
        eulbfs_solver* h = sl.s;
        double* part = (double*)(h->ws + h->L.red_partial);
        double* dout = (double*)(h->ws + h->L.red_out);
        HIP_TRY(launch_reduce<R>(h->dp, state_at<R>(h->ws, h->L.W0, h->L), part, h->L.red_blocks, dout, b->stream));
        HIP_TRY(hipMemcpyAsync(b->h_sums + (size_t)k * NRED, dout, NRED * sizeof(double), hipMemcpyDeviceToHost,
                               b->stream));
    }
    HIP_TRY(hipEventCreateWithFlags(&te.ev, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(te.ev, b->stream));
    te.tick = b->tick;
    b->events.push_back(te);
    for (int k : act) {
        Slot& sl = b->slots[k];
        sl.done += s_eff;
        sl.s->steps += s_eff;
        if (sl.done >= sl.nsteps) sl.finish_tick = b->tick;
    }
    ++b->tick;
    return EULBFS_OK;
}

// Copy n doubles of host planes to dst (device) through the batch's pinned
// staging buffer on the upload stream; the batch stream waits for the copy.
int admit_stage(eulbfs_batch* b, const double* src, size_t n, char* dst)
{
    std::string* err = &b->err;
    HIP_TRY(hipEventSynchronize(b->stage_done));  // the previous upload has left the buffer
    if (b->stage_cap < n) {
        if (b->h_stage) HIP_TRY(hipHostFree(b->h_stage));
        b->h_stage = nullptr;
        b->stage_cap = 0;
        HIP_TRY(hipHostMalloc((void**)&b->h_stage, n * sizeof(double), hipHostMallocDefault));
        b->stage_cap = n;
    }
    std::memcpy(b->h_stage, src, n * sizeof(double));
    HIP_TRY(hipMemcpyAsync(dst, b->h_stage, n * sizeof(double), hipMemcpyHostToDevice, b->upload));
    HIP_TRY(hipEventRecord(b->stage_done, b->upload));
    HIP_TRY(hipStreamWaitEvent(b->stream, b->stage_done, 0));
    return EULBFS_OK;
}

// The request's last tick has completed: nothing enqueued touches it any more.
bool slot_settled(eulbfs_batch* b, const Slot& sl)
{
    batch_progress(b, false);
    return sl.done >= sl.nsteps && sl.finish_tick >= 0 && sl.finish_tick < b->completed_tick;
}

Slot* batch_slot(eulbfs_batch* b, int32_t slot)
{
    if (!b || slot < 0 || slot >= b->max_slots || !b->slots[slot].s) return nullptr;
    return &b->slots[slot];
}

}  // namespace

extern "C" {

size_t eulbfs_batch_request_bytes(const eulbfs_params* prm)
{
    if (!check(prm).empty()) return 0;
    const eulbfs_params p = batch_view(prm);
    return align_up(make_layout(&p).total);
}

int eulbfs_batch_create(size_t hbm_budget, int32_t max_slots, int32_t precision, void* d_ws, size_t ws_bytes,
                        void* hip_stream, eulbfs_batch_t* out)
{
    std::string* err = nullptr;
    if (!out) return set_err(err, EULBFS_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_slots <= 0 || max_slots > 65536) return set_err(err, EULBFS_EINVAL, "max_slots must be in 1..65536");
    if (precision != EULBFS_FP64 && precision != EULBFS_FP32) return set_err(err, EULBFS_EINVAL, "unknown precision");
    if (hbm_budget < ((size_t)1 << 20)) return set_err(err, EULBFS_EINVAL, "hbm_budget below 1 MiB");
    eulbfs_batch* b = new eulbfs_batch();
    b->budget = hbm_budget;
    b->max_slots = max_slots;
    b->precision = precision;
    b->stream = (hipStream_t)hip_stream;
    b->slots.resize(max_slots);
    b->desc_bytes = align_up((size_t)max_slots * desc_size(precision));
    // a whole tile holds 512 cells (either shape) of at least 88 bytes (three
    // FP32-mode copies of W + dF_s/dt); partial tiles at the grids' edges get
    // as much again
    static_assert(BATCH_TX[0] * BATCH_TY[0] == 512 && BATCH_TX[1] * BATCH_TY[1] == 512, "512-cell batch tiles");
    b->tile_cap = 2 * (max_slots + (int)std::min<size_t>(hbm_budget / ((size_t)512 * 88), 1 << 25));
    const size_t tiles_bytes = align_up((size_t)b->tile_cap * sizeof(int));
    const size_t tables = 2 * (b->desc_bytes + tiles_bytes);
    if (hbm_budget <= tables) {
        delete b;
        return set_err(err, EULBFS_EINVAL, "hbm_budget too small for the batch tables");
    }
    if (d_ws) {
        if (ws_bytes < hbm_budget || ((uintptr_t)d_ws % ALIGN) != 0) {
            delete b;
            return set_err(err, EULBFS_EINVAL, "workspace must be >= hbm_budget bytes and 256-byte aligned");
        }
        b->base = (char*)d_ws;
    } else {
        const hipError_t e = hipMalloc(&b->base, hbm_budget);
        if (e != hipSuccess) {
            delete b;
            return set_err(err, EULBFS_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        }
        b->own = true;
    }
    char* p = b->base;
    for (int k = 0; k < 2; ++k) {
        b->d_desc[k] = p;
        p += b->desc_bytes;
        b->d_tiles[k] = (int*)p;
        p += tiles_bytes;
    }
    b->arena = p;
    b->arena_bytes = hbm_budget - tables;
    b->free_list.push_back({0, b->arena_bytes});
    bool ok = true;
    for (int k = 0; k < 2 && ok; ++k) {
        ok &= hipHostMalloc((void**)&b->h_desc[k], b->desc_bytes, hipHostMallocDefault) == hipSuccess;
        ok &= hipHostMalloc((void**)&b->h_tiles[k], tiles_bytes, hipHostMallocDefault) == hipSuccess;
        ok &= hipEventCreateWithFlags(&b->upload_done[k], hipEventDisableTiming) == hipSuccess;
    }
    ok = ok && hipHostMalloc((void**)&b->h_sums, (size_t)max_slots * NRED * sizeof(double), hipHostMallocDefault) ==
                   hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&b->upload, hipStreamNonBlocking) == hipSuccess;  // default priority
    ok = ok && hipEventCreateWithFlags(&b->stage_done, hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        eulbfs_batch_destroy(b);
        return set_err(err, EULBFS_EDEVICE, "batch set-up failed (pinned tables, streams or events)");
    }
    *out = b;
    return EULBFS_OK;
}

int eulbfs_batch_admit(eulbfs_batch_t b, const eulbfs_params* prm, const eulbfs_init* init, int64_t nsteps,
                       int32_t* slot)
{
    if (!b) return set_err(nullptr, EULBFS_EINVAL, "batch is NULL");
    std::string* err = &b->err;
    if (!slot) return set_err(err, EULBFS_EINVAL, "slot is NULL");
    *slot = -1;
    const std::string e = check(prm);
    if (!e.empty()) return set_err(err, EULBFS_EINVAL, e);
    if (prm->precision != b->precision) return set_err(err, EULBFS_EINVAL, "request precision differs from the batch");
    if (nsteps <= 0) return set_err(err, EULBFS_EINVAL, "nsteps must be > 0");
    int k = 0;
    while (k < b->max_slots && b->slots[k].s) ++k;
    if (k == b->max_slots) return set_err(err, EULBFS_EBUSY, "no free slot");
    const std::string ie = init_error(init);
    if (!ie.empty()) return set_err(err, EULBFS_EINVAL, ie);
    const eulbfs_params p = batch_view(prm);
    const Layout L = make_layout(&p);
    const size_t bytes = align_up(L.total);
    const size_t off = arena_alloc(b, bytes);
    if (off == SIZE_MAX) return set_err(err, EULBFS_EBUSY, "not enough free arena for this request");
    // Host planes go through pinned memory and the upload stream into the
    // request's own staging area (its arena range is idle: a freed range is
    // only reused once its last tick has completed), so admission does not
    // wait for the ticks in flight; the batch stream waits for the copy.
    if (L.mesh_bytes) {  // stretched mesh: its tables take the same route
        const std::vector<double> t = mesh_tables(&p, L);
        const int rc = admit_stage(b, t.data(), t.size(), b->arena + off + L.mesh);
        if (rc != EULBFS_OK) {
            arena_free(b, off, bytes);
            return rc;
        }
    }
    eulbfs_init dinit = *init;
    if (init->kind != EULBFS_INIT_ANALYTIC && !init->on_device) {
        const size_t n6 = (size_t)6 * p.nx * p.ny;
        int rc = admit_stage(b, init->planes, n6, b->arena + off + L.staging);
        if (rc != EULBFS_OK) {
            arena_free(b, off, bytes);
            return rc;
        }
        dinit.on_device = 1;
        dinit.planes = (const double*)(b->arena + off + L.staging);
    }
    eulbfs_solver* h = nullptr;
    const int rc = create_solver(&p, &dinit, b->arena + off, bytes, b->stream, false, &h);
    if (rc != EULBFS_OK) {
        arena_free(b, off, bytes);
        return set_err(err, rc, g_thread_err);
    }
    Slot& sl = b->slots[k];
    sl.s = h;
    sl.serial = b->admitted++;
    sl.off = off;
    sl.bytes = bytes;
    sl.nsteps = nsteps;
    sl.done = 0;
    sl.finish_tick = -1;
    *slot = k;
    return EULBFS_OK;
}

int eulbfs_batch_tick(eulbfs_batch_t b, int32_t steps)
{
    if (!b) return set_err(nullptr, EULBFS_EINVAL, "batch is NULL");
    if (steps <= 0) return set_err(&b->err, EULBFS_EINVAL, "steps must be > 0");
    return b->precision == EULBFS_FP32 ? batch_tick<float>(b, steps) : batch_tick<double>(b, steps);
}

int eulbfs_batch_poll(eulbfs_batch_t b, int32_t* done, int32_t cap, int32_t* n)
{
    if (!b) return set_err(nullptr, EULBFS_EINVAL, "batch is NULL");
    if (!n || (cap > 0 && !done)) return set_err(&b->err, EULBFS_EINVAL, "bad output arguments");
    batch_progress(b, false);
    int cnt = 0;
    for (int k = 0; k < b->max_slots && cnt < cap; ++k) {
        const Slot& sl = b->slots[k];
        if (sl.s && sl.done >= sl.nsteps && sl.finish_tick >= 0 && sl.finish_tick < b->completed_tick)
            done[cnt++] = k;
    }
    *n = cnt;
    return EULBFS_OK;
}

int eulbfs_batch_query(eulbfs_batch_t b, int32_t slot, int32_t what, void* out, size_t bytes, int32_t out_on_device)
{
    Slot* sl = batch_slot(b, slot);
    if (!sl) return set_err(b ? &b->err : nullptr, EULBFS_EINVAL, "no request in this slot");
    if (what == EULBFS_SCALAR_DIAG && !out_on_device && out && bytes >= EULBFS_NDIAG * sizeof(double) &&
        slot_settled(b, *sl)) {  // summed by the finishing tick: no wait
        diag_from_sums(sl->s, b->h_sums + (size_t)slot * NRED, (double*)out);
        const std::string why = unstable_reason((const double*)out);
        if (!why.empty()) {
            sl->s->poisoned = true;
            return set_err(&b->err, EULBFS_EUNSTABLE, why + " at the end of the request");
        }
        return EULBFS_OK;
    }
    const int rc = eulbfs_query(sl->s, what, out, bytes, out_on_device);
    if (rc != EULBFS_OK) b->err = sl->s->err;
    return rc;
}

int eulbfs_batch_release(eulbfs_batch_t b, int32_t slot)
{
    Slot* sl = batch_slot(b, slot);
    if (!sl) return set_err(b ? &b->err : nullptr, EULBFS_EINVAL, "no request in this slot");
    // an unfinished request's planes may still be in use by enqueued launches
    const bool settled = slot_settled(b, *sl);
    if (!settled) (void)hipStreamSynchronize(b->stream);
    free_solver(sl->s, false);
    arena_free(b, sl->off, sl->bytes);
    *sl = Slot();
    return EULBFS_OK;
}

int eulbfs_batch_set_tile(eulbfs_batch_t b, int32_t tile)
{
    if (!b) return set_err(nullptr, EULBFS_EINVAL, "batch is NULL");
    if (tile < EULBFS_BATCH_TILE_AUTO || tile > NBATCH_TILES)
        return set_err(&b->err, EULBFS_EINVAL, "unknown batch tile");
    b->tile_mode = tile;
    return EULBFS_OK;
}

int eulbfs_batch_schedule(eulbfs_batch_t b, eulbfs_batch_sched* out)
{
    static_assert(NBATCH_TILES == 2 && EULBFS_BATCH_TILE_64x8 == NBATCH_TILES, "the header's two batch tiles");
    if (!b) return set_err(nullptr, EULBFS_EINVAL, "batch is NULL");
    if (!out) return set_err(&b->err, EULBFS_EINVAL, "out is NULL");
    batch_progress(b, false);
    *out = eulbfs_batch_sched{};
    out->next_tile = batch_pick_tile(b) + 1;
    for (int k = 0; k < NBATCH_TILES; ++k) {
        out->ns_per_cell_step[k] = b->tile_cells[k] > 0.0 ? 1e6 * b->tile_ms[k] / b->tile_cells[k] : 0.0;
        out->ticks_timed[k] = b->tile_ticks[k];
    }
    out->time_ratio = b->pairs ? std::exp(b->log_ratio) : 0.0;
    out->pairs = b->pairs;
    return EULBFS_OK;
}

int eulbfs_batch_destroy(eulbfs_batch_t b)
{
    if (!b) return EULBFS_OK;
    (void)hipStreamSynchronize(b->stream);
    if (b->upload) (void)hipStreamSynchronize(b->upload);
    for (auto& sl : b->slots)
        if (sl.s) free_solver(sl.s, false);
    for (auto& te : b->events) {
        (void)hipEventDestroy(te.ev);
        if (te.t0) (void)hipEventDestroy(te.t0);
        if (te.t1) (void)hipEventDestroy(te.t1);
    }
    if (b->h_sums) (void)hipHostFree(b->h_sums);
    if (b->h_stage) (void)hipHostFree(b->h_stage);
    if (b->stage_done) (void)hipEventDestroy(b->stage_done);
    if (b->upload) (void)hipStreamDestroy(b->upload);
    for (int k = 0; k < 2; ++k) {
        if (b->h_desc[k]) (void)hipHostFree(b->h_desc[k]);
        if (b->h_tiles[k]) (void)hipHostFree(b->h_tiles[k]);
        if (b->upload_done[k]) (void)hipEventDestroy(b->upload_done[k]);
    }
    for (int k = 0; k < 2; ++k)
        if (b->step_graph[k]) (void)hipGraphExecDestroy(b->step_graph[k]);
    if (b->own && b->base) (void)hipFree(b->base);
    delete b;
    return EULBFS_OK;
}

const char* eulbfs_batch_last_error(eulbfs_batch_t b)
{
    if (!b) return g_thread_err.c_str();
    return b->err.c_str();
}

}  // extern "C"
