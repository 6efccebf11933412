// HIP kernels of the EULBFS time step for gfx950 (MI355X).
//
//   k_stage_fused   one SSP-RK3 stage (Eq. 58) of a whole grid: a 2-D tile of
//                   cells per workgroup stages W of the tile plus three halo
//                   layers in LDS (boundary rules applied on the fly at the
//                   domain edge), recovers the primitive fields (Eqs. 5-7),
//                   mu_c, computes every face flux of the tile once (Eqs.
//                   53-56), then updates its cells with the sources of Eq. (51),
//                   the RK combination and the momentum projection.
//   k_stage_batched the same tile body over the tiles of every grid of a batch.
//   k_fill_ghosts / k_split_prims / k_split_faces / k_split_update
//                   the same stage in four kernels with the intermediate
//                   fields in HBM (ghosted state, primitive planes, face flux
//                   planes); used for face-by-face checks and as a variant.
// Each stage kernel has a stretched-mesh variant (template flag NU) that takes
// the geometry from per-column and per-row tables instead of one dx.
//   k_init          primitive initial fields -> conserved vector.
//   k_export        conserved or derived field -> dense double plane.
//   k_reduce_*      FP64 integrals, deterministic two-pass wave reduction.
#include <algorithm>

#include "eulbfs_device.h"
#include "eulbfs_internal.h"

namespace eulbfs {

// ---------------------------------------------------------------------------
// Per-cell update shared by the fused and the split stage kernels: Wk is the
// cell's stage input, Wnk its W^n (the same values in the first stage), fsd
// its lagged dF_s/dt.
// ---------------------------------------------------------------------------
template <typename R, int FAST = 0>
__device__ __forceinline__ void cell_update(const DevParams& P, const StageCoef& K, const R c[NPRIM + 1],
                                            const Cons<R>& Wk, const Cons<R>& Wnk, R fsd, R dudx, R dvdy,
                                            R drhodx, R drhody, R dmudx, R dmudy, const R dF[5],
                                            const State<R>& out, R* fsdot, R* resid, size_t resid_stride, size_t q)
{
    R Fl = R(0);
    if (P.surf_model == 1) {
        double fl, T;
        closure<FAST>(P, Wk.H, clamp01(Wk.C), fl, T);
        Fl = R(fl);
    }
    R S[5];
    sources<R, FAST>(P, c, Fl, fsd, dudx, dvdy, drhodx, drhody, dmudx, dmudy, S);
    R res[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) res[k] = -dF[k] + S[k];
    if (resid) {
#pragma unroll
        for (int k = 0; k < 5; ++k) resid[k * resid_stride + q] = res[k];
        return;
    }
    const Cons<R>& wn = Wnk;
    const double cdt = K.cc * P.dt;
    const double Hnew = K.ca * wn.H + K.cb * Wk.H + cdt * (double)res[0];
    // FP32 fields: the stage combination as W^n plus its increment,
    // W^n + b (W^(k) - W^n) + c dt R (a + b = 1 in every stage), so p and M
    // are rounded once relative to their value and otherwise only relative to
    // the (small) increment; a W^n + b W^(k) + c dt R in FP32 rounded three
    // times relative to the value and let a near-steady field drift
    R pnew, mxnew, mynew;
    if constexpr (sizeof(R) == sizeof(float)) {
        const R cb = R(K.cb), cdtr = R(cdt);
        pnew = wn.p + (cb * (Wk.p - wn.p) + cdtr * res[1]);
        mxnew = wn.mx + (cb * (Wk.mx - wn.mx) + cdtr * res[2]);
        mynew = wn.my + (cb * (Wk.my - wn.my) + cdtr * res[3]);
    } else {
        const R ca = R(K.ca), cb = R(K.cb), cdtr = R(cdt);
        pnew = ca * wn.p + cb * Wk.p + cdtr * res[1];
        mxnew = ca * wn.mx + cb * Wk.mx + cdtr * res[2];
        mynew = ca * wn.my + cb * Wk.my + cdtr * res[3];
    }
    const double Cnew = K.ca * wn.C + K.cb * Wk.C + cdt * (double)res[4];
    // rigid solid: M <- (1 - F_s) M with F_s of the new stage value
    const double Fs_new = solid_fraction<FAST>(P, Hnew, Cnew);
    mxnew *= R(1.0 - Fs_new);
    mynew *= R(1.0 - Fs_new);
    // streaming stores: the next stage reads these values on other CUs, so
    // keeping them out of the writing XCD's L2 spares the write-back at the
    // end of the launch (2 % faster at 512 x 512)
    __builtin_nontemporal_store(Hnew, &out.H[q]);
    __builtin_nontemporal_store(pnew, &out.p[q]);
    __builtin_nontemporal_store(mxnew, &out.mx[q]);
    __builtin_nontemporal_store(mynew, &out.my[q]);
    __builtin_nontemporal_store(Cnew, &out.C[q]);
    if (K.last) __builtin_nontemporal_store(R((Fs_new - solid_fraction<FAST>(P, wn.H, wn.C)) * P.inv_dt), &fsdot[q]);
}

// ---------------------------------------------------------------------------
// Fused stage kernel.
//
// LDS: the W tile with three halo layers is only needed until the primitive
// fields exist, so the face fluxes reuse its bytes; the primitive planes
// (tile + two halo layers) live through the whole stage.  The density plane
// is stored when it fits in the 160 KB of a CU; otherwise (32 x 32 in FP64)
// rho is recomputed from C and F_s where it is read, by the same expression
// as in primitives(), so both forms give the same bits.
// ---------------------------------------------------------------------------
constexpr size_t LDS_PER_CU = 160 * 1024;

template <typename R, int TX, int TY>
struct FusedLds {
    static constexpr int W3 = TX + 2 * NG, H3 = TY + 2 * NG;
    static constexpr int W2 = TX + 4, H2 = TY + 4;
    static constexpr int NFX = (TX + 1) * TY, NFY = TX * (TY + 1);
    static constexpr size_t BYTES_W = (size_t)W3 * H3 * (2 * sizeof(double) + 3 * sizeof(R));
    static constexpr size_t BYTES_F = (size_t)5 * (NFX + NFY) * sizeof(R);
    static constexpr size_t BYTES_U = BYTES_W > BYTES_F ? BYTES_W : BYTES_F;
    static constexpr bool RHO = BYTES_U + (size_t)(NPRIM + 1) * W2 * H2 * sizeof(R) <= LDS_PER_CU;
    static constexpr int NPL = RHO ? NPRIM + 1 : NPRIM;  // stored primitive planes
};

// Density of a primitive-plane entry (Eq. 7 with the clamped C and F_s).
template <typename R, bool RHO, int N>
__device__ __forceinline__ R plane_rho(const DevParams& P, const R (*sP)[N], int q)
{
    if constexpr (RHO) return sP[NPRIM][q];
    else return mix<R>(P.rho, clamp01(sP[VC][q]), sP[VFS][q]);
}

// Derivative weights (MESH_GM, MESH_G0, MESH_GP) of ghosted index l.
template <typename R>
__device__ __forceinline__ void mesh_grad(const double* m, int stride, int l, R c[3])
{
    c[0] = R(m[MESH_GM * stride + l]);
    c[1] = R(m[MESH_G0 * stride + l]);
    c[2] = R(m[MESH_GP * stride + l]);
}

// One tile of one stage: cells [i0, i0+TX) x [j0, j0+TY) of the grid described
// by P.  Every thread of the workgroup must call it (it synchronises).  NU:
// stretched mesh, the geometry read from the mesh tables of P (ghosted column
// and row indices clamped to the table's valid range; only cells beyond the
// ghost ring of a partial tile are clamped, and their results are never
// stored).
template <typename R, int LAT, int FAST, int TX, int TY, bool NU = false>
__device__ __forceinline__ void stage_tile(const DevParams& P, const StageCoef& K, const State<R>& in,
                                           const State<R>& Wn, const State<R>& out, R* fsdot, int i0, int j0)
{
    using L = FusedLds<R, TX, TY>;
    constexpr int NT = TX * TY;
    constexpr int W3 = L::W3, H3 = L::H3, W2 = L::W2, H2 = L::H2, NFX = L::NFX, NFY = L::NFY;
    __shared__ __align__(16) char sU[L::BYTES_U];
    constexpr bool RHO = L::RHO;
    __shared__ R sP[L::NPL][W2 * H2];
    double* sH = reinterpret_cast<double*>(sU);                                // H, then C
    double* sC = sH + W3 * H3;
    R* sW = reinterpret_cast<R*>(sU + (size_t)2 * W3 * H3 * sizeof(double));  // p, Mx, My
    R* sF = reinterpret_cast<R*>(sU);                                          // 5 planes of NFX+NFY

    const int tid = threadIdx.x;
    // NU: the mesh weights (MESH_*) of the W2 columns and H2 rows of the tile
    // and two halo layers, staged once per tile in FP64 (mu_c is formed in
    // FP64 whatever the field type)
    constexpr int NMW = NU ? NMESH * (W2 + H2) : 1;
    __shared__ double sMesh[NMW];
    auto mx = [&](int k, int li) { return sMesh[k * W2 + li]; };
    auto my = [&](int k, int lj) { return sMesh[NMESH * W2 + k * H2 + lj]; };
    // ghosted column / row index of the tile + 2 layers (li, lj in [0, W2)),
    // clamped to the rows of the tables that hold derivative weights
    auto gcol = [&](int li) { return min(i0 + li + 1, P.nx + 2 * NG - 2); };
    auto grow = [&](int lj) { return min(j0 + lj + 1, P.ny + 2 * NG - 2); };
    __syncthreads();  // the LDS of a previous tile of this workgroup is free
    if constexpr (NU) {
        for (int t = tid; t < NMW; t += NT) {
            if (t < NMESH * W2)
                sMesh[t] = P.mxc[(t / W2) * P.msx + gcol(t % W2)];
            else
                sMesh[t] = P.myc[((t - NMESH * W2) / H2) * P.msy + grow((t - NMESH * W2) % H2)];
        }
    }

    // 1. stage W of the tile and three halo layers (boundary rules only for
    // tiles whose halo leaves the grid)
    auto stage = [&](int q, const Cons<R>& w) {
        sH[q] = w.H;
        sW[0 * W3 * H3 + q] = w.p;
        sW[1 * W3 * H3 + q] = w.mx;
        sW[2 * W3 * H3 + q] = w.my;
        sC[q] = w.C;
    };
    // every load of a thread is issued before the first LDS store, so the
    // memory latency is paid once rather than once per pass
    constexpr int NQ = W3 * H3, NIT = (NQ + NT - 1) / NT;
    Cons<R> w[NIT];
    if (i0 >= NG && j0 >= NG && i0 + TX + NG <= P.nx && j0 + TY + NG <= P.ny) {
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int q = tid + it * NT;
            if (q < NQ) w[it] = read_cell(in, P.pitch, i0 + q % W3 - NG, j0 + q / W3 - NG);
        }
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int q = tid + it * NT;
            if (q < NQ) stage(q, w[it]);
        }
    } else {
        // Tiles whose halo leaves the grid, in the order of load_bc (which the
        // split path uses) and with its values: (a) cells of the grid and
        // periodic images, plain loads; (b) x-wall ghosts of the rows that are
        // not y-wall ghosts; (c) y-wall ghosts of every column.  A ghost's
        // mirror and first interior cells lie inside the tile, so (b) and (c)
        // read them from LDS.  Positions beyond the ghost ring are clamped onto
        // it first, as in load_bc.
        auto cl = [](int g, int n) { return min(max(g, -NG), n + NG - 1); };
        bool inside[NIT];
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int q = tid + it * NT;
            int gi = cl(i0 + q % W3 - NG, P.nx), gj = cl(j0 + q / W3 - NG, P.ny);
            if (P.periodic_x) gi = wrap(gi, P.nx);
            if (P.periodic_y) gj = wrap(gj, P.ny);
            inside[it] = q < NQ && gi >= 0 && gi < P.nx && gj >= 0 && gj < P.ny;
            if (inside[it]) w[it] = read_cell(in, P.pitch, gi, gj);
        }
#pragma unroll
        for (int it = 0; it < NIT; ++it)
            if (inside[it]) stage(tid + it * NT, w[it]);
        auto cons_at = [&](int q) {
            Cons<R> c;
            c.H = sH[q];
            c.p = sW[q];
            c.mx = sW[W3 * H3 + q];
            c.my = sW[2 * W3 * H3 + q];
            c.C = sC[q];
            return c;
        };
        // one wall rule for the ghost at clamped normal index g (outside
        // [0, n)); base: LDS index of normal index 0 on the ghost's line,
        // stride: LDS step along the normal
        auto ghost = [&](int side, int g, int n, int base, int stride) {
            const bool lo = g < 0;
            const int k = lo ? -g : g - n + 1;
            const int m = lo ? k - 1 : n - k, first = lo ? 0 : n - 1, dir = lo ? 1 : -1;
            const int qm = base + m * stride, qf = base + first * stride;
            const double Cw = sC[qf];
            double wet;
            if (NU)
                wet = P.hyst[side] ? wet_factor_nu(P, side, Cw, sC[qf + dir * stride], sC[qf + 2 * dir * stride])
                                   : P.mside[side * MS_STRIDE + MS_WET];
            else
                wet = P.hyst[side] ? wet_factor(P, side, Cw, sC[qf + dir * stride], sC[qf + 2 * dir * stride])
                                   : P.wet[side];
            return wall_ghost<R, NU>(P, side, k, cons_at(qm), Cw, wet);
        };
        __syncthreads();
        // One thread per ghost cell, the ghost columns (rows) of one side at a
        // time: the side is a loop constant, so each wall's constants are
        // scalar loads, and most tiles need a single pass of the first waves.
        // Ghost columns of a side: LDS columns [0, NG - i0) below the wall at
        // 0, [nx - i0 + NG, W3) beyond the wall at nx (the latter includes the
        // columns past the ring of a partial tile).
        if (!P.periodic_x) {
            for (int sd = 0; sd < 2; ++sd) {
                const int c0 = sd == 0 ? 0 : P.nx - i0 + NG;
                const int nc = sd == 0 ? max(0, NG - i0) : max(0, W3 - c0);
                for (int c = tid; c < nc * H3; c += NT) {
                    const int lj = c / nc, li = c0 + c % nc;
                    const int gi = cl(i0 + li - NG, P.nx), gj = cl(j0 + lj - NG, P.ny);
                    if (P.periodic_y || (gj >= 0 && gj < P.ny))
                        stage(lj * W3 + li, ghost(sd, gi, P.nx, lj * W3 + NG - i0, 1));
                }
            }
            __syncthreads();
        }
        if (!P.periodic_y) {
            for (int sd = 2; sd < 4; ++sd) {
                const int r0 = sd == 2 ? 0 : P.ny - j0 + NG;
                const int nr = sd == 2 ? max(0, NG - j0) : max(0, H3 - r0);
                for (int c = tid; c < nr * W3; c += NT) {
                    const int lj = r0 + c / W3, li = c % W3;
                    const int gj = cl(j0 + lj - NG, P.ny);
                    stage(lj * W3 + li, ghost(sd, gj, P.ny, (NG - j0) * W3 + li, W3));
                }
            }
        }
    }
    __syncthreads();

    // 2. primitives and mu_c on the tile and two halo layers
    for (int q = tid; q < W2 * H2; q += NT) {
        const int li = q % W2, lj = q / W2;
        const int q3 = (lj + 1) * W3 + li + 1;
        Cons<R> w;
        w.H = sH[q3];
        w.p = sW[q3];
        w.mx = sW[W3 * H3 + q3];
        w.my = sW[2 * W3 * H3 + q3];
        w.C = sC[q3];
        R pr[NPRIM + 1];
        primitives<R, FAST>(P, w, pr);
        if (NU) {  // chem_potential_nu with the staged weights
            const double lap = mx(MESH_LM, li) * sC[q3 - 1] + mx(MESH_L0, li) * w.C + mx(MESH_LP, li) * sC[q3 + 1] +
                               my(MESH_LM, lj) * sC[q3 - W3] + my(MESH_L0, lj) * w.C + my(MESH_LP, lj) * sC[q3 + W3];
            pr[VMU] = R(2.0 * P.beta * w.C * (w.C - 1.0) * (2.0 * w.C - 1.0) - P.kappa * lap);
        } else
            pr[VMU] = R(chem_potential(P, w.C, sC[q3 + 1], sC[q3 - 1], sC[q3 + W3], sC[q3 - W3]));
#pragma unroll
        for (int k = 0; k < L::NPL; ++k) sP[k][q] = pr[k];
    }
    __syncthreads();

    // 3. every face of the tile once (fluxes overwrite the dead W tile).  The
    // x faces are padded to whole waves in the iteration space, so every wave
    // takes either the x or the y branch in a pass, never both.
    const R i2dx = R(P.inv_2dx);
    const R c_sh = R(0.5 * P.dx - P.delta_t) * i2dx, c_h = R(0.5 * P.dx) * i2dx, c_ds = R(P.delta_t) * i2dx;
    const R ds = R(P.delta_t);
    constexpr int NF = NFX + NFY;
    constexpr int NFXP = (NFX + 63) / 64 * 64;
    static_assert(NT % 64 == 0, "whole waves per workgroup");
    // A SIMD issues from its oldest ready wave first, so the oldest waves of a
    // workgroup finish their faces early and the youngest run the end of the
    // pass alone.  With one 1024-thread workgroup per CU a wave's priority
    // drops with each face it has done, which keeps the waves of a SIMD abreast
    // (2-5 % faster).  Where several workgroups share a CU the raised priority
    // starves the others' loads instead (10-15 % slower), so smaller tiles
    // keep the default.
    constexpr bool PRIO = NT >= 1024;
    // tiles with a wall face (uniform over the workgroup: interior tiles skip
    // the per-face test)
    const bool wall_x = !P.periodic_x && (i0 == 0 || i0 + TX >= P.nx);
    const bool wall_y = !P.periodic_y && (j0 == 0 || j0 + TY >= P.ny);
    if (PRIO) __builtin_amdgcn_s_setprio(3);
    for (int fp = tid; fp < NFXP + NFY; fp += NT) {
        if (PRIO && fp != tid) {
            if (fp < tid + 2 * NT) __builtin_amdgcn_s_setprio(2);
            else __builtin_amdgcn_s_setprio(1);
        }
        if (fp >= NFX && fp < NFXP) continue;  // padding of the x faces
        const int f = fp < NFXP ? fp : fp - NFXP + NFX;  // storage index: x faces, then y faces
        Bases<R> X;
        R F[5];
        if (f < NFX) {
            const int fi = f % (TX + 1), fj = f / (TX + 1);
            const int a = (fj + 2) * W2 + fi + 1;
            if (NU) {
                const R ca[3] = {R(mx(MESH_GM, fi + 1)), R(mx(MESH_G0, fi + 1)), R(mx(MESH_GP, fi + 1))};
                const R cb[3] = {R(mx(MESH_GM, fi + 2)), R(mx(MESH_G0, fi + 2)), R(mx(MESH_GP, fi + 2))};
                const R ct[3] = {R(my(MESH_GM, fj + 2)), R(my(MESH_G0, fj + 2)), R(my(MESH_GP, fj + 2))};
                const R ha = R(mx(MESH_HW, fi + 1)), hb = R(mx(MESH_HW, fi + 2));
#pragma unroll
                for (int k = 0; k < NPRIM; ++k)
                    face_bases_nu(sP[k], a, 1, W2, ca, cb, ct, ha, hb, ds, X.A[k], X.B[k], X.M[k], X.da[k],
                                  X.db[k], X.dm[k]);
            } else {
#pragma unroll
                for (int k = 0; k < NPRIM; ++k)
                    face_bases<R, FAST>(sP[k], a, 1, W2, c_sh, c_h, c_ds, X.A[k], X.B[k], X.M[k], X.da[k],
                                        X.db[k], X.dm[k]);
            }
            X.rho_a = plane_rho<R, RHO>(P, sP, a);
            X.rho_b = plane_rho<R, RHO>(P, sP, a + 1);
            face_flux<R, LAT, FAST>(P, X, F);
            const int gi = i0 + fi;
            if (wall_x) {
                if (gi == 0) wall_face(P, 0, F);
                else if (gi == P.nx) wall_face(P, 1, F);
            }
#pragma unroll
            for (int k = 0; k < 5; ++k) sF[k * NF + f] = F[k];
        } else {
            const int g = f - NFX;
            const int fi = g % TX, fj = g / TX;
            const int a = (fj + 1) * W2 + fi + 2;
            if (NU) {
                const R ca[3] = {R(my(MESH_GM, fj + 1)), R(my(MESH_G0, fj + 1)), R(my(MESH_GP, fj + 1))};
                const R cb[3] = {R(my(MESH_GM, fj + 2)), R(my(MESH_G0, fj + 2)), R(my(MESH_GP, fj + 2))};
                const R ct[3] = {R(mx(MESH_GM, fi + 2)), R(mx(MESH_G0, fi + 2)), R(mx(MESH_GP, fi + 2))};
                const R ha = R(my(MESH_HW, fj + 1)), hb = R(my(MESH_HW, fj + 2));
#pragma unroll
                for (int k = 0; k < NPRIM; ++k) {
                    const int ks = k == VU ? VV : (k == VV ? VU : k);  // local frame n = y, t = x
                    face_bases_nu(sP[ks], a, W2, 1, ca, cb, ct, ha, hb, ds, X.A[k], X.B[k], X.M[k], X.da[k],
                                  X.db[k], X.dm[k]);
                }
            } else {
#pragma unroll
                for (int k = 0; k < NPRIM; ++k) {
                    const int ks = k == VU ? VV : (k == VV ? VU : k);  // local frame n = y, t = x
                    face_bases<R, FAST>(sP[ks], a, W2, 1, c_sh, c_h, c_ds, X.A[k], X.B[k], X.M[k], X.da[k],
                                        X.db[k], X.dm[k]);
                }
            }
            X.rho_a = plane_rho<R, RHO>(P, sP, a);
            X.rho_b = plane_rho<R, RHO>(P, sP, a + W2);
            face_flux<R, LAT, FAST>(P, X, F);
            const int gj = j0 + fj;
            if (wall_y) {
                if (gj == 0) wall_face(P, 2, F);
                else if (gj == P.ny) wall_face(P, 3, F);
            }
            sF[0 * NF + f] = F[0];
            sF[1 * NF + f] = F[1];
            sF[2 * NF + f] = F[3];  // x-momentum flux through a y-face: sum e_y e_x f*
            sF[3 * NF + f] = F[2];
            sF[4 * NF + f] = F[4];
        }
    }
    if (PRIO) __builtin_amdgcn_s_setprio(0);
    // 4. cell update.  The cell's stage input, W^n and dF_s/dt are loaded
    // before the barrier: a wave that is done with its faces waits for them
    // while the last faces are computed.
    const int tx = tid % TX, ty = tid / TX;
    const int i = i0 + tx, j = j0 + ty;
    const bool own = i < P.nx && j < P.ny;
    const size_t q = (size_t)j * P.pitch + i;
    Cons<R> wk{}, wnk{};
    R fsd = R(0);
    if (own) {
        wk = read_cell(in, P.pitch, i, j);
        wnk = read_at(Wn, q);
        fsd = fsdot[q];
    }
    __syncthreads();
    if (!own) return;  // no barrier follows in this tile
    const int fl = ty * (TX + 1) + tx;
    const int fb = NFX + ty * TX + tx;
    // Eq. (52) on a Cartesian cell: (1/V) S = 1/width along each direction
    const R idx = NU ? R(mx(MESH_IW, tx + 2)) : R(P.inv_dx);
    const R idy = NU ? R(my(MESH_IW, ty + 2)) : idx;
    R dF[5];
#pragma unroll
    for (int k = 0; k < 5; ++k)
        dF[k] = (sF[k * NF + fl + 1] - sF[k * NF + fl]) * idx + (sF[k * NF + fb + TX] - sF[k * NF + fb]) * idy;
    const int c2 = (ty + 2) * W2 + tx + 2;
    R c[NPRIM + 1];
#pragma unroll
    for (int k = 0; k < NPRIM; ++k) c[k] = sP[k][c2];
    c[NPRIM] = plane_rho<R, RHO>(P, sP, c2);
    R dudx, dvdy, drx, dry, dmx, dmy;
    if (NU) {
        const R gx[3] = {R(mx(MESH_GM, tx + 2)), R(mx(MESH_G0, tx + 2)), R(mx(MESH_GP, tx + 2))};
        const R gy[3] = {R(my(MESH_GM, ty + 2)), R(my(MESH_G0, ty + 2)), R(my(MESH_GP, ty + 2))};
        dudx = gx[0] * sP[VU][c2 - 1] + gx[1] * sP[VU][c2] + gx[2] * sP[VU][c2 + 1];
        dvdy = gy[0] * sP[VV][c2 - W2] + gy[1] * sP[VV][c2] + gy[2] * sP[VV][c2 + W2];
        drx = gx[0] * plane_rho<R, RHO>(P, sP, c2 - 1) + gx[1] * c[NPRIM] + gx[2] * plane_rho<R, RHO>(P, sP, c2 + 1);
        dry = gy[0] * plane_rho<R, RHO>(P, sP, c2 - W2) + gy[1] * c[NPRIM] +
              gy[2] * plane_rho<R, RHO>(P, sP, c2 + W2);
        dmx = gx[0] * sP[VMU][c2 - 1] + gx[1] * sP[VMU][c2] + gx[2] * sP[VMU][c2 + 1];
        dmy = gy[0] * sP[VMU][c2 - W2] + gy[1] * sP[VMU][c2] + gy[2] * sP[VMU][c2 + W2];
    } else {
        dudx = (sP[VU][c2 + 1] - sP[VU][c2 - 1]) * i2dx;
        dvdy = (sP[VV][c2 + W2] - sP[VV][c2 - W2]) * i2dx;
        drx = (plane_rho<R, RHO>(P, sP, c2 + 1) - plane_rho<R, RHO>(P, sP, c2 - 1)) * i2dx;
        dry = (plane_rho<R, RHO>(P, sP, c2 + W2) - plane_rho<R, RHO>(P, sP, c2 - W2)) * i2dx;
        dmx = (sP[VMU][c2 + 1] - sP[VMU][c2 - 1]) * i2dx;
        dmy = (sP[VMU][c2 + W2] - sP[VMU][c2 - W2]) * i2dx;
    }
    cell_update<R, FAST>(P, K, c, wk, wnk, fsd, dudx, dvdy, drx, dry, dmx, dmy, dF, out, fsdot, (R*)nullptr, 0, q);
}

// One stage of one grid.  Workgroups are dispatched round-robin over the
// eight XCDs of the chip, each with its own L2; giving every XCD a
// contiguous run of tiles keeps the halo rows a tile shares with its
// neighbours in the same L2.
template <typename R, int LAT, int FAST, int TX, int TY, bool NU = false>
__global__ void __launch_bounds__(TX* TY)
    k_stage_fused(DevParams P, StageCoef K, State<R> in, State<R> Wn, State<R> out, R* fsdot, int tiles_x,
                  int ntiles, int per_xcd)
{
    const int b = blockIdx.x;
    const int t = (b % NXCD) * per_xcd + b / NXCD;
    if (t >= ntiles) return;
    stage_tile<R, LAT, FAST, TX, TY, NU>(P, K, in, Wn, out, fsdot, (t % tiles_x) * TX, (t / tiles_x) * TY);
}

// One stage of every grid of a batch: one workgroup per tile of the
// concatenated tile list of all resident requests (tile_req maps a tile to
// its request), so one launch covers grids of any size mix.  Consecutive
// tiles go to one XCD, as in k_stage_fused.  (A persistent grid looping over
// the tiles held more registers per thread, one wave fewer per SIMD in FP32,
// and ran 20-30 % slower.)
template <typename R, int LAT, int FAST, int TX, int TY, bool NU = false>
__global__ void __launch_bounds__(TX* TY)
    k_stage_batched(const BatchDesc<R>* __restrict__ descs, const int* __restrict__ tile_req, int ntiles,
                    StageCoef K, int stage)
{
    const int per_xcd = (ntiles + NXCD - 1) / NXCD;
    const int b = blockIdx.x;
    const int t = (b % NXCD) * per_xcd + b / NXCD;
    if (t >= ntiles) return;
    const BatchDesc<R>& D = descs[tile_req[t]];
    const int lt = t - D.tile0;  // tile index within its request, 0 <= lt < tiles of the request
    const State<R>& in = D.W[stage];
    const State<R>& out = D.W[stage == 2 ? 0 : stage + 1];
    stage_tile<R, LAT, FAST, TX, TY, NU>(D.P, K, in, D.W[0], out, D.fsdot, (lt % D.tiles_x) * TX,
                                         (lt / D.tiles_x) * TY);
}

// ---------------------------------------------------------------------------
// Split path.  Ghosted planes have (ny + 6) rows of gpitch elements; cell
// (i, j) sits at (j + 3) * gpitch + i + 3.  NU: stretched mesh (the geometry
// comes from the mesh tables of DevParams instead of dx).
// ---------------------------------------------------------------------------
template <typename R, bool NU>
__global__ void k_fill_ghosts(DevParams P, State<R> in, State<R> g, int gpitch)
{
    const int li = blockIdx.x * blockDim.x + threadIdx.x;
    const int lj = blockIdx.y * blockDim.y + threadIdx.y;
    if (li >= P.nx + 2 * NG || lj >= P.ny + 2 * NG) return;
    const Cons<R> w = load_bc<R, NU>(P, in, li - NG, lj - NG);
    const size_t q = (size_t)lj * gpitch + li;
    g.H[q] = w.H;
    g.p[q] = w.p;
    g.mx[q] = w.mx;
    g.my[q] = w.my;
    g.C[q] = w.C;
}

template <typename R, bool NU>
__global__ void k_split_prims(DevParams P, State<R> g, int gpitch, R* prim, size_t pstride)
{
    const int li = blockIdx.x * blockDim.x + threadIdx.x + 1;  // ring 2 of the ghosted grid
    const int lj = blockIdx.y * blockDim.y + threadIdx.y + 1;
    if (li >= P.nx + 2 * NG - 1 || lj >= P.ny + 2 * NG - 1) return;
    const size_t q = (size_t)lj * gpitch + li;
    Cons<R> w;
    w.H = g.H[q];
    w.p = g.p[q];
    w.mx = g.mx[q];
    w.my = g.my[q];
    w.C = g.C[q];
    R pr[NPRIM + 1];
    primitives(P, w, pr);
    if (NU)
        pr[VMU] = R(chem_potential_nu(P, li, lj, w.C, g.C[q + 1], g.C[q - 1], g.C[q + gpitch], g.C[q - gpitch]));
    else
        pr[VMU] = R(chem_potential(P, w.C, g.C[q + 1], g.C[q - 1], g.C[q + gpitch], g.C[q - gpitch]));
#pragma unroll
    for (int k = 0; k <= NPRIM; ++k) prim[k * pstride + q] = pr[k];
}

// The split kernels launch 64x4 threads; the bound lets the face and update
// kernels keep their bases and coefficients in registers (the default bound of
// 1024 threads caps a wave at 128 VGPRs, and the stretched-mesh variants spilled).
constexpr int SPLIT_THREADS = 256;

template <typename R, int LAT, bool NU>
__global__ void __launch_bounds__(SPLIT_THREADS) k_split_faces(DevParams P, const R* prim, size_t pstride, int gpitch, R* Fx, R* Fy, int fpitch,
                              size_t fstride)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const R i2dx = R(P.inv_2dx);
    const R c_sh = R(0.5 * P.dx - P.delta_t) * i2dx, c_h = R(0.5 * P.dx) * i2dx, c_ds = R(P.delta_t) * i2dx;
    const R ds = R(P.delta_t);
    Bases<R> X;
    R F[5];
    if (i <= P.nx && j < P.ny) {  // x-face i between cells i-1 and i
        const int a = (j + NG) * gpitch + (i - 1 + NG);
        R ca[3], cb[3], ct[3], ha = 0, hb = 0;
        if (NU) {
            mesh_grad(P.mxc, P.msx, i - 1 + NG, ca);
            mesh_grad(P.mxc, P.msx, i + NG, cb);
            mesh_grad(P.myc, P.msy, j + NG, ct);
            ha = R(P.mxc[MESH_HW * P.msx + i - 1 + NG]);
            hb = R(P.mxc[MESH_HW * P.msx + i + NG]);
        }
#pragma unroll
        for (int k = 0; k < NPRIM; ++k) {
            if (NU)
                face_bases_nu(prim + k * pstride, a, 1, gpitch, ca, cb, ct, ha, hb, ds, X.A[k], X.B[k], X.M[k],
                              X.da[k], X.db[k], X.dm[k]);
            else
                face_bases(prim + k * pstride, a, 1, gpitch, c_sh, c_h, c_ds, X.A[k], X.B[k], X.M[k], X.da[k],
                           X.db[k], X.dm[k]);
        }
        face_flux<R, LAT>(P, X, F);
        if (!P.periodic_x) {
            if (i == 0) wall_face(P, 0, F);
            else if (i == P.nx) wall_face(P, 1, F);
        }
        const size_t o = (size_t)j * fpitch + i;
#pragma unroll
        for (int k = 0; k < 5; ++k) Fx[k * fstride + o] = F[k];
    }
    if (i < P.nx && j <= P.ny) {  // y-face j between cells j-1 and j
        const int a = (j - 1 + NG) * gpitch + (i + NG);
        R ca[3], cb[3], ct[3], ha = 0, hb = 0;
        if (NU) {
            mesh_grad(P.myc, P.msy, j - 1 + NG, ca);
            mesh_grad(P.myc, P.msy, j + NG, cb);
            mesh_grad(P.mxc, P.msx, i + NG, ct);
            ha = R(P.myc[MESH_HW * P.msy + j - 1 + NG]);
            hb = R(P.myc[MESH_HW * P.msy + j + NG]);
        }
#pragma unroll
        for (int k = 0; k < NPRIM; ++k) {
            const int ks = k == VU ? VV : (k == VV ? VU : k);
            if (NU)
                face_bases_nu(prim + ks * pstride, a, gpitch, 1, ca, cb, ct, ha, hb, ds, X.A[k], X.B[k], X.M[k],
                              X.da[k], X.db[k], X.dm[k]);
            else
                face_bases(prim + ks * pstride, a, gpitch, 1, c_sh, c_h, c_ds, X.A[k], X.B[k], X.M[k], X.da[k],
                           X.db[k], X.dm[k]);
        }
        face_flux<R, LAT>(P, X, F);
        if (!P.periodic_y) {
            if (j == 0) wall_face(P, 2, F);
            else if (j == P.ny) wall_face(P, 3, F);
        }
        const size_t o = (size_t)j * fpitch + i;
        Fy[0 * fstride + o] = F[0];
        Fy[1 * fstride + o] = F[1];
        Fy[2 * fstride + o] = F[3];
        Fy[3 * fstride + o] = F[2];
        Fy[4 * fstride + o] = F[4];
    }
}

template <typename R, bool NU>
__global__ void __launch_bounds__(SPLIT_THREADS) k_split_update(DevParams P, StageCoef K, const R* prim, size_t pstride, int gpitch, const R* Fx,
                               const R* Fy, int fpitch, size_t fstride, State<R> in, State<R> Wn, State<R> out,
                               R* fsdot, R* resid, size_t resid_stride)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= P.nx || j >= P.ny) return;
    // Eq. (52) on a Cartesian cell: (1/V) S = 1/width along each direction
    const R idx = NU ? R(P.mxc[MESH_IW * P.msx + i + NG]) : R(P.inv_dx);
    const R idy = NU ? R(P.myc[MESH_IW * P.msy + j + NG]) : idx;
    const size_t o = (size_t)j * fpitch + i;
    R dF[5];
#pragma unroll
    for (int k = 0; k < 5; ++k)
        dF[k] = (Fx[k * fstride + o + 1] - Fx[k * fstride + o]) * idx +
                (Fy[k * fstride + o + fpitch] - Fy[k * fstride + o]) * idy;
    const size_t c2 = (size_t)(j + NG) * gpitch + i + NG;
    R c[NPRIM + 1];
#pragma unroll
    for (int k = 0; k <= NPRIM; ++k) c[k] = prim[k * pstride + c2];
    const R i2dx = R(P.inv_2dx);
    const R* pu = prim + VU * pstride;
    const R* pv = prim + VV * pstride;
    const R* pr = prim + NPRIM * pstride;
    const R* pm = prim + VMU * pstride;
    R dudx, dvdy, drx, dry, dmx, dmy;
    if (NU) {
        R gx[3], gy[3];
        mesh_grad(P.mxc, P.msx, i + NG, gx);
        mesh_grad(P.myc, P.msy, j + NG, gy);
        auto ddx = [&](const R* v) { return gx[0] * v[c2 - 1] + gx[1] * v[c2] + gx[2] * v[c2 + 1]; };
        auto ddy = [&](const R* v) { return gy[0] * v[c2 - gpitch] + gy[1] * v[c2] + gy[2] * v[c2 + gpitch]; };
        dudx = ddx(pu);
        dvdy = ddy(pv);
        drx = ddx(pr);
        dry = ddy(pr);
        dmx = ddx(pm);
        dmy = ddy(pm);
    } else {
        dudx = (pu[c2 + 1] - pu[c2 - 1]) * i2dx;
        dvdy = (pv[c2 + gpitch] - pv[c2 - gpitch]) * i2dx;
        drx = (pr[c2 + 1] - pr[c2 - 1]) * i2dx;
        dry = (pr[c2 + gpitch] - pr[c2 - gpitch]) * i2dx;
        dmx = (pm[c2 + 1] - pm[c2 - 1]) * i2dx;
        dmy = (pm[c2 + gpitch] - pm[c2 - gpitch]) * i2dx;
    }
    const size_t q = (size_t)j * P.pitch + i;
    const Cons<R> wk = read_cell(in, P.pitch, i, j);
    const Cons<R> wnk = read_at(Wn, q);
    cell_update(P, K, c, wk, wnk, fsdot[q], dudx, dvdy, drx, dry, dmx, dmy, dF, out, fsdot, resid, resid_stride, q);
}

// ---------------------------------------------------------------------------
// Initial state, export, set
// ---------------------------------------------------------------------------
template <typename R>
__global__ void k_init(DevParams P, const double* prim6, State<R> out, R* fsdot)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= P.nx || j >= P.ny) return;
    const size_t n = (size_t)P.nx * P.ny, s = (size_t)j * P.nx + i;
    const double T = prim6[s], Fl = prim6[n + s], C = prim6[2 * n + s];
    const double u = prim6[3 * n + s], v = prim6[4 * n + s], p = prim6[5 * n + s];
    const double H = enthalpy_of(P, T, Fl, C);
    const double Cc = clamp01(C);
    const double Fs = solid_fraction(P, H, C);
    const double rho = mix<double>(P.rho, Cc, Fs);
    const size_t q = (size_t)j * P.pitch + i;
    out.H[q] = H;
    out.p[q] = R(p);
    out.mx[q] = R(rho / 3.0 * u);
    out.my[q] = R(rho / 3.0 * v);
    out.C[q] = C;
    fsdot[q] = R(0);
}

// The n-th output of the splitmix64 generator with state seed (Steele, Lea
// and Flood, OOPSLA 2014): state seed + n 0x9E3779B97F4A7C15 through the
// generator's output mix; the top 53 bits as a number uniform in [-1, 1).
__device__ __forceinline__ double splitmix_uniform(uint64_t seed, uint64_t n)
{
    uint64_t z = seed + n * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1.0p-52 - 1.0;
}

// Cell centre along one direction, the first face at 0: the running sum of
// the widths up to and including cell i, in index order, less half the
// cell's own width.  hw: the tabulated half widths (stretched mesh; twice a
// half width is the width exactly) or nullptr (every width dx).
__device__ __forceinline__ double cell_centre(const double* hw, int i, double dx)
{
    double c = 0.0;
    for (int k = 0; k <= i; ++k) c += hw ? 2.0 * hw[k] : dx;
    return c - (hw ? hw[i] : 0.5 * dx);
}

// Closed-form primitive fields T, F_l, C, u, v, p (six dense planes).
__global__ void k_init_shape(DevParams P, InitShape S, double* prim6)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= P.nx || j >= P.ny) return;
    const size_t n = (size_t)P.nx * P.ny, s = (size_t)j * P.nx + i;
    const double* hwx = P.mside ? P.mxc + MESH_HW * P.msx + NG : nullptr;
    const double* hwy = P.mside ? P.myc + MESH_HW * P.msy + NG : nullptr;
    // one rounding per operation, as the closed forms are written (no fused
    // multiply-adds across these statements)
    double C = S.c0;
    if (S.profile == 1) {
        const double c = S.axis == 0 ? cell_centre(hwx, i, P.dx) : cell_centre(hwy, j, P.dx);
        const double d = 2.0 * (S.h0 - c);
        C = 0.5 * (1.0 + tanh(d / S.xi));
    } else if (S.profile == 2) {
        const double dx = cell_centre(hwx, i, P.dx) - S.x0, dy = cell_centre(hwy, j, P.dx) - S.y0;
        const double dx2 = dx * dx, dy2 = dy * dy;
        const double d = 2.0 * (S.r0 - sqrt(dx2 + dy2));
        C = 0.5 * (1.0 + tanh(d / S.xi));
    }
    double T = C > 0.5 ? S.t_in : S.t_out;
    if (S.t_amp != 0.0) {
        const double noise = S.t_amp * splitmix_uniform(S.seed, (uint64_t)s + 1);
        T = T + noise;
    }
    prim6[s] = T;
    prim6[n + s] = S.fl0;
    prim6[2 * n + s] = C;
    prim6[3 * n + s] = S.u_in != 0.0 ? S.u_in * C : 0.0;
    prim6[4 * n + s] = S.v_in != 0.0 ? S.v_in * C : 0.0;
    prim6[5 * n + s] = 0.0;
}

template <typename R>
__global__ void k_set_conserved(DevParams P, const double* w6, State<R> out, R* fsdot, int which)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= P.nx || j >= P.ny) return;
    const size_t n = (size_t)P.nx * P.ny, s = (size_t)j * P.nx + i;
    const size_t q = (size_t)j * P.pitch + i;
    // which: -1 all six planes, else one plane (0..5) read from w6[0..n)
    for (int k = 0; k < 6; ++k) {
        if (which >= 0 && k != which) continue;
        const double x = which >= 0 ? w6[s] : w6[k * n + s];
        switch (k) {
            case 0: out.H[q] = x; break;
            case 1: out.p[q] = R(x); break;
            case 2: out.mx[q] = R(x); break;
            case 3: out.my[q] = R(x); break;
            case 4: out.C[q] = x; break;
            default: fsdot[q] = R(x); break;
        }
    }
}

template <typename R>
__global__ void k_export(DevParams P, State<R> S, const R* fsdot, int what, double* dst)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= P.nx || j >= P.ny) return;
    const size_t q = (size_t)j * P.pitch + i, s = (size_t)j * P.nx + i;
    const Cons<R> w = read_cell(S, P.pitch, i, j);
    double x = 0.0;
    if (what <= 5) {
        switch (what) {
            case 0: x = w.H; break;
            case 1: x = w.p; break;
            case 2: x = w.mx; break;
            case 3: x = w.my; break;
            case 4: x = w.C; break;
            default: x = fsdot[q]; break;
        }
    } else if (what == 12) {
        if (P.mside) {
            const double cE = load_bc<R, true>(P, S, i + 1, j).C, cW = load_bc<R, true>(P, S, i - 1, j).C;
            const double cN = load_bc<R, true>(P, S, i, j + 1).C, cS = load_bc<R, true>(P, S, i, j - 1).C;
            x = chem_potential_nu(P, i + NG, j + NG, w.C, cE, cW, cN, cS);
        } else {
            const double cE = load_bc(P, S, i + 1, j).C, cW = load_bc(P, S, i - 1, j).C;
            const double cN = load_bc(P, S, i, j + 1).C, cS = load_bc(P, S, i, j - 1).C;
            x = chem_potential(P, w.C, cE, cW, cN, cS);
        }
    } else {
        const double Cc = clamp01(w.C);
        double Fl, T;
        closure(P, w.H, Cc, Fl, T);
        const double Fs = Cc * (1.0 - Fl);
        const double rho = (double)mix<R>(P.rho, R(Cc), R(Fs));
        switch (what) {
            case 6: x = T; break;
            case 7: x = Fl; break;
            case 8: x = Fs; break;
            case 9: x = rho; break;
            case 10: x = (double)(w.mx * (R(3) / R(rho))); break;
            default: x = (double)(w.my * (R(3) / R(rho))); break;
        }
    }
    dst[s] = x;
}

template <typename R>
__global__ void k_export_ghosted(DevParams P, State<R> S, double* dst, int gnx, int gny)
{
    const int li = blockIdx.x * blockDim.x + threadIdx.x;
    const int lj = blockIdx.y * blockDim.y + threadIdx.y;
    if (li >= gnx || lj >= gny) return;
    const Cons<R> w = P.mside ? load_bc<R, true>(P, S, li - NG, lj - NG) : load_bc(P, S, li - NG, lj - NG);
    const size_t n = (size_t)gnx * gny, s = (size_t)lj * gnx + li;
    dst[s] = w.H;
    dst[n + s] = w.p;
    dst[2 * n + s] = w.mx;
    dst[3 * n + s] = w.my;
    dst[4 * n + s] = w.C;
}

// ---------------------------------------------------------------------------
// Deterministic FP64 reductions: per-block partials in a fixed order, then
// one block sums the partials in a fixed order.
// ---------------------------------------------------------------------------
constexpr int RED_THREADS = 256;

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// partial layout: [block][NRED] (RED_* slots); RED_UMAX, RED_NEG_CMIN and
// RED_CMAX are maxima, the others sums.  The order parameter's extremes start
// at -1e300 so that a block without cells leaves them out of the maxima.
__device__ __forceinline__ constexpr bool red_is_max(int k)
{
    return k == RED_UMAX || k == RED_NEG_CMIN || k == RED_CMAX;
}

__device__ __forceinline__ void red_init(double acc[NRED])
{
#pragma unroll
    for (int k = 0; k < NRED; ++k) acc[k] = k == RED_NEG_CMIN || k == RED_CMAX ? -1e300 : 0.0;
}

template <typename R>
__global__ void __launch_bounds__(RED_THREADS) k_reduce_partial(DevParams P, State<R> S, double* partial)
{
    __shared__ double sred[RED_THREADS / 64][NRED];
    double acc[NRED];
    red_init(acc);
    const size_t n = (size_t)P.nx * P.ny;
    const int ic = P.nx / 2;
    for (size_t s = (size_t)blockIdx.x * RED_THREADS + threadIdx.x; s < n; s += (size_t)gridDim.x * RED_THREADS) {
        const int i = (int)(s % P.nx), j = (int)(s / P.nx);
        const Cons<R> w = read_cell(S, P.pitch, i, j);
        const double Cc = clamp01(w.C);
        double Fl, T;
        closure(P, w.H, Cc, Fl, T);
        const double Fs = Cc * (1.0 - Fl);
        const double rho = mix<double>(P.rho, Cc, Fs);
        const double u = 3.0 * (double)w.mx / rho, v = 3.0 * (double)w.my / rho;
        // stretched mesh: cell volume and height inside the sums (uniform: dx^2 and dx after them)
        const double hy = P.mside ? 2.0 * P.myc[MESH_HW * P.msy + j + NG] : 1.0;
        const double wx = P.mside ? 2.0 * P.mxc[MESH_HW * P.msx + i + NG] : 1.0;
        const double dV = wx * hy;
        acc[RED_RHO] += rho * dV;
        acc[RED_C] += w.C * dV;
        acc[RED_H] += w.H * dV;
        acc[RED_FS] += Fs * dV;
        acc[RED_UMAX] = fmax(acc[RED_UMAX], sqrt(u * u + v * v));
        const bool finite = isfinite(w.H) && isfinite((double)w.p) && isfinite((double)w.mx) &&
                            isfinite((double)w.my) && isfinite(w.C);
        acc[RED_NONFINITE] += finite ? 0.0 : 1.0;
        acc[RED_NEG_CMIN] = fmax(acc[RED_NEG_CMIN], -w.C);
        acc[RED_CMAX] = fmax(acc[RED_CMAX], w.C);
        if (i == ic) {
            acc[RED_TIP] += Fs * hy;
            acc[RED_AXIS] += Cc * hy;
        }
        if (j == 0) acc[RED_WALL] += Cc * wx;
    }
    const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
#pragma unroll
    for (int k = 0; k < NRED; ++k) {
        const double r = red_is_max(k) ? wave_max(acc[k]) : wave_sum(acc[k]);
        if (lane == 0) sred[wv][k] = r;
    }
    __syncthreads();
    if (threadIdx.x < NRED) {
        const int k = threadIdx.x;
        double r = sred[0][k];
        for (int w = 1; w < RED_THREADS / 64; ++w) r = red_is_max(k) ? fmax(r, sred[w][k]) : r + sred[w][k];
        partial[(size_t)blockIdx.x * NRED + k] = r;
    }
}

__global__ void __launch_bounds__(RED_THREADS) k_reduce_final(const double* partial, int nblocks, double* out)
{
    __shared__ double sred[RED_THREADS / 64][NRED];
    double acc[NRED];
    red_init(acc);
    for (int b = threadIdx.x; b < nblocks; b += RED_THREADS)
        for (int k = 0; k < NRED; ++k)
            acc[k] = red_is_max(k) ? fmax(acc[k], partial[(size_t)b * NRED + k]) : acc[k] + partial[(size_t)b * NRED + k];
    const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
#pragma unroll
    for (int k = 0; k < NRED; ++k) {
        const double r = red_is_max(k) ? wave_max(acc[k]) : wave_sum(acc[k]);
        if (lane == 0) sred[wv][k] = r;
    }
    __syncthreads();
    if (threadIdx.x < NRED) {
        const int k = threadIdx.x;
        double r = sred[0][k];
        for (int w = 1; w < RED_THREADS / 64; ++w) r = red_is_max(k) ? fmax(r, sred[w][k]) : r + sred[w][k];
        out[k] = r;
    }
}

// ---------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------
static inline dim3 grid2(int nx, int ny, dim3 b) { return dim3((nx + b.x - 1) / b.x, (ny + b.y - 1) / b.y); }

template <typename R, int LAT, int FAST, int TX, int TY, bool NU = false>
static hipError_t launch_fused_t(const DevParams& P, const StageCoef& K, const State<R>& in, const State<R>& Wn,
                                 const State<R>& out, R* fsdot, hipStream_t st)
{
    const int tiles_x = (P.nx + TX - 1) / TX, tiles_y = (P.ny + TY - 1) / TY;
    const int ntiles = tiles_x * tiles_y;
    const int per_xcd = (ntiles + NXCD - 1) / NXCD;
    hipLaunchKernelGGL((k_stage_fused<R, LAT, FAST, TX, TY, NU>), dim3(per_xcd * NXCD), dim3(TX * TY), 0, st, P, K,
                       in, Wn, out, fsdot, tiles_x, ntiles, per_xcd);
    return hipGetLastError();
}

// Stretched meshes: one tile shape per field type (NuTile) and no FAST_HALF
// (delta_t is not half of every width).
template <typename R, int LAT>
static hipError_t launch_fused_nu(const DevParams& P, const StageCoef& K, const State<R>& in, const State<R>& Wn,
                                  const State<R>& out, R* fsdot, hipStream_t st)
{
    constexpr int TX = NuTile<R>::TX, TY = NuTile<R>::TY;
    if (P.fast & FAST_UCP) return launch_fused_t<R, LAT, FAST_UCP, TX, TY, true>(P, K, in, Wn, out, fsdot, st);
    return launch_fused_t<R, LAT, 0, TX, TY, true>(P, K, in, Wn, out, fsdot, st);
}

template <typename R, int LAT, int FAST>
static hipError_t launch_fused_f(const DevParams& P, int tile, const StageCoef& K, const State<R>& in,
                                 const State<R>& Wn, const State<R>& out, R* fsdot, hipStream_t st)
{
    switch (tile) {
        case TILE_16x16: return launch_fused_t<R, LAT, FAST, 16, 16>(P, K, in, Wn, out, fsdot, st);
        case TILE_64x8: return launch_fused_t<R, LAT, FAST, 64, 8>(P, K, in, Wn, out, fsdot, st);
        case TILE_64x4: return launch_fused_t<R, LAT, FAST, 64, 4>(P, K, in, Wn, out, fsdot, st);
        case TILE_32x16: return launch_fused_t<R, LAT, FAST, 32, 16>(P, K, in, Wn, out, fsdot, st);
        case TILE_32x32: return launch_fused_t<R, LAT, FAST, 32, 32>(P, K, in, Wn, out, fsdot, st);
        default: return launch_fused_t<R, LAT, FAST, 32, 8>(P, K, in, Wn, out, fsdot, st);
    }
}

template <typename R, int LAT>
static hipError_t launch_fused_l(const DevParams& P, int tile, const StageCoef& K, const State<R>& in,
                                 const State<R>& Wn, const State<R>& out, R* fsdot, hipStream_t st)
{
    switch (P.fast & (FAST_HALF | FAST_UCP)) {
        case FAST_HALF: return launch_fused_f<R, LAT, FAST_HALF>(P, tile, K, in, Wn, out, fsdot, st);
        case FAST_UCP: return launch_fused_f<R, LAT, FAST_UCP>(P, tile, K, in, Wn, out, fsdot, st);
        case FAST_HALF | FAST_UCP:
            return launch_fused_f<R, LAT, FAST_HALF | FAST_UCP>(P, tile, K, in, Wn, out, fsdot, st);
        default: return launch_fused_f<R, LAT, 0>(P, tile, K, in, Wn, out, fsdot, st);
    }
}

template <typename R>
hipError_t launch_stage_fused(const DevParams& P, int tile, const StageCoef& K, const State<R>& in,
                              const State<R>& Wn, const State<R>& out, R* fsdot, hipStream_t st)
{
    if (P.mside) {
        if (P.lattice_hg == 5) return launch_fused_nu<R, 5>(P, K, in, Wn, out, fsdot, st);
        return launch_fused_nu<R, 9>(P, K, in, Wn, out, fsdot, st);
    }
    if (P.lattice_hg == 5) return launch_fused_l<R, 5>(P, tile, K, in, Wn, out, fsdot, st);
    return launch_fused_l<R, 9>(P, tile, K, in, Wn, out, fsdot, st);
}

template <typename R, int LAT, int FAST, int TB, bool NU = false>
static void launch_batched_t(const BatchDesc<R>* descs, const int* tile_req, int ntiles, const StageCoef& K,
                             int stage, hipStream_t st)
{
    constexpr int TX = BATCH_TX[TB], TY = BATCH_TY[TB];
    const int per_xcd = (ntiles + NXCD - 1) / NXCD;
    hipLaunchKernelGGL((k_stage_batched<R, LAT, FAST, TX, TY, NU>), dim3(per_xcd * NXCD), dim3(TX * TY), 0, st,
                       descs, tile_req, ntiles, K, stage);
}

template <typename R, int LAT, int TB>
static void launch_batched_f(const BatchDesc<R>* descs, const int* tile_req, int ntiles, int f, const StageCoef& K,
                             int stage, hipStream_t st)
{
    switch (f) {
        case FAST_HALF: launch_batched_t<R, LAT, FAST_HALF, TB>(descs, tile_req, ntiles, K, stage, st); break;
        case FAST_UCP: launch_batched_t<R, LAT, FAST_UCP, TB>(descs, tile_req, ntiles, K, stage, st); break;
        case FAST_HALF | FAST_UCP:
            launch_batched_t<R, LAT, FAST_HALF | FAST_UCP, TB>(descs, tile_req, ntiles, K, stage, st);
            break;
        default: launch_batched_t<R, LAT, 0, TB>(descs, tile_req, ntiles, K, stage, st); break;
    }
}

// Requests of one batched launch share the mesh kind, the lattice and the
// fast-path flags (a stretched mesh never has FAST_HALF); tile indexes
// BATCH_TX/BATCH_TY and is the one their tile list was built for (stretched
// meshes: always 0).
template <typename R>
hipError_t launch_stage_batched(const BatchDesc<R>* descs, const int* tile_req, int ntiles, int lattice, int fast,
                                bool nu, int tile, const StageCoef& K, int stage, hipStream_t st)
{
    if (ntiles <= 0) return hipSuccess;
    const int f = fast & (FAST_HALF | FAST_UCP);
    if (nu) {
        const bool ucp = (f & FAST_UCP) != 0;
        if (lattice == 5) {
            if (ucp) launch_batched_t<R, 5, FAST_UCP, 0, true>(descs, tile_req, ntiles, K, stage, st);
            else launch_batched_t<R, 5, 0, 0, true>(descs, tile_req, ntiles, K, stage, st);
        } else {
            if (ucp) launch_batched_t<R, 9, FAST_UCP, 0, true>(descs, tile_req, ntiles, K, stage, st);
            else launch_batched_t<R, 9, 0, 0, true>(descs, tile_req, ntiles, K, stage, st);
        }
        return hipGetLastError();
    }
    if (lattice == 5) {
        if (tile == 1) launch_batched_f<R, 5, 1>(descs, tile_req, ntiles, f, K, stage, st);
        else launch_batched_f<R, 5, 0>(descs, tile_req, ntiles, f, K, stage, st);
    } else {
        if (tile == 1) launch_batched_f<R, 9, 1>(descs, tile_req, ntiles, f, K, stage, st);
        else launch_batched_f<R, 9, 0>(descs, tile_req, ntiles, f, K, stage, st);
    }
    return hipGetLastError();
}

template <typename R, bool NU>
hipError_t split_stages(const DevParams& P, const SplitScratch<R>& X, const StageCoef& K, const State<R>& in,
                        const State<R>& Wn, const State<R>& out, R* fsdot, R* resid, size_t resid_stride,
                        hipStream_t st)
{
    const dim3 b(64, SPLIT_THREADS / 64);
    hipLaunchKernelGGL((k_fill_ghosts<R, NU>), grid2(P.nx + 2 * NG, P.ny + 2 * NG, b), b, 0, st, P, in, X.g,
                       X.gpitch);
    hipLaunchKernelGGL((k_split_prims<R, NU>), grid2(P.nx + 4, P.ny + 4, b), b, 0, st, P, X.g, X.gpitch, X.prim,
                       X.pstride);
    if (P.lattice_hg == 5)
        hipLaunchKernelGGL((k_split_faces<R, 5, NU>), grid2(P.nx + 1, P.ny + 1, b), b, 0, st, P, (const R*)X.prim,
                           X.pstride, X.gpitch, X.Fx, X.Fy, X.fpitch, X.fstride);
    else
        hipLaunchKernelGGL((k_split_faces<R, 9, NU>), grid2(P.nx + 1, P.ny + 1, b), b, 0, st, P, (const R*)X.prim,
                           X.pstride, X.gpitch, X.Fx, X.Fy, X.fpitch, X.fstride);
    hipLaunchKernelGGL((k_split_update<R, NU>), grid2(P.nx, P.ny, b), b, 0, st, P, K, (const R*)X.prim, X.pstride,
                       X.gpitch, (const R*)X.Fx, (const R*)X.Fy, X.fpitch, X.fstride, in, Wn, out, fsdot, resid,
                       resid_stride);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_stage_split(const DevParams& P, const SplitScratch<R>& X, const StageCoef& K, const State<R>& in,
                              const State<R>& Wn, const State<R>& out, R* fsdot, R* resid, size_t resid_stride,
                              hipStream_t st)
{
    if (P.mside) return split_stages<R, true>(P, X, K, in, Wn, out, fsdot, resid, resid_stride, st);
    return split_stages<R, false>(P, X, K, in, Wn, out, fsdot, resid, resid_stride, st);
}

template <typename R>
hipError_t launch_init(const DevParams& P, const double* prim6, const State<R>& out, R* fsdot, hipStream_t st)
{
    const dim3 b(64, 4);
    hipLaunchKernelGGL(k_init<R>, grid2(P.nx, P.ny, b), b, 0, st, P, prim6, out, fsdot);
    return hipGetLastError();
}

hipError_t launch_init_shape(const DevParams& P, const InitShape& S, double* prim6, hipStream_t st)
{
    const dim3 b(64, 4);
    hipLaunchKernelGGL(k_init_shape, grid2(P.nx, P.ny, b), b, 0, st, P, S, prim6);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_set_conserved(const DevParams& P, const double* w6, const State<R>& out, R* fsdot, int which,
                                hipStream_t st)
{
    const dim3 b(64, 4);
    hipLaunchKernelGGL(k_set_conserved<R>, grid2(P.nx, P.ny, b), b, 0, st, P, w6, out, fsdot, which);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_export(const DevParams& P, const State<R>& S, const R* fsdot, int what, double* dst,
                         hipStream_t st)
{
    const dim3 b(64, 4);
    if (what == 14) {
        hipLaunchKernelGGL(k_export_ghosted<R>, grid2(P.nx + 2 * NG, P.ny + 2 * NG, b), b, 0, st, P, S, dst,
                           P.nx + 2 * NG, P.ny + 2 * NG);
    } else {
        hipLaunchKernelGGL(k_export<R>, grid2(P.nx, P.ny, b), b, 0, st, P, S, fsdot, what, dst);
    }
    return hipGetLastError();
}

template <typename R>
hipError_t launch_reduce(const DevParams& P, const State<R>& S, double* partial, int nblocks, double* out,
                         hipStream_t st)
{
    hipLaunchKernelGGL(k_reduce_partial<R>, dim3(nblocks), dim3(RED_THREADS), 0, st, P, S, partial);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(RED_THREADS), 0, st, (const double*)partial, nblocks, out);
    return hipGetLastError();
}

#define EULBFS_INSTANTIATE(R)                                                                                      \
    template hipError_t launch_stage_fused<R>(const DevParams&, int, const StageCoef&, const State<R>&,            \
                                              const State<R>&, const State<R>&, R*, hipStream_t);                  \
    template hipError_t launch_stage_split<R>(const DevParams&, const SplitScratch<R>&, const StageCoef&,          \
                                              const State<R>&, const State<R>&, const State<R>&, R*, R*, size_t,   \
                                              hipStream_t);                                                        \
    template hipError_t launch_init<R>(const DevParams&, const double*, const State<R>&, R*, hipStream_t);         \
    template hipError_t launch_set_conserved<R>(const DevParams&, const double*, const State<R>&, R*, int,         \
                                                hipStream_t);                                                      \
    template hipError_t launch_export<R>(const DevParams&, const State<R>&, const R*, int, double*, hipStream_t);  \
    template hipError_t launch_reduce<R>(const DevParams&, const State<R>&, double*, int, double*, hipStream_t);   \
    template hipError_t launch_stage_batched<R>(const BatchDesc<R>*, const int*, int, int, int, bool, int,         \
                                                const StageCoef&, int, hipStream_t);

EULBFS_INSTANTIATE(double)
EULBFS_INSTANTIATE(float)

}  // namespace eulbfs
