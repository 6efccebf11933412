"""Mutation check of the oracle pins (run by hand; not collected by pytest).

Each entry plants one plausible mistake in a copy of oracle/eulbfs_oracle.c
(a flipped sign, a dropped term, a swapped index or operand), builds it, and
runs tests/test_oracle_pins.py and tests/test_oracle_mesh.py against it.  Every mutant must make at least
one pin fail.

    python tests/oracle_mutants.py [name ...]
"""
import os, shutil, subprocess, sys, tempfile
SRC = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MUTS = {
 'mesh_d1_central': ('return (hm * hm * (vp - v0) + hp * hp * (v0 - vm)) / (hm * hp * (hm + hp));', 'return (vp - vm) / (hm + hp);'),
 'mesh_d2_width': ('return 2.0 * ((vp - v0) / hp - (v0 - vm) / hm) / (hm + hp);', 'return ((vp - v0) / hp - (v0 - vm) / hm) / hm;'),
 'mesh_hxm': ('return 0.5 * (WX(g, i - 1) + WX(g, i)); }', 'return 0.5 * (WX(g, i + 1) + WX(g, i)); }'),
 'mesh_half_swap': ('0.5 * WX(g, i - 1), 0.5 * WX(g, i), F);', '0.5 * WX(g, i), 0.5 * WX(g, i - 1), F);'),
 'mesh_residual_width': ('-dfx / WX(g, i) - dfy / WY(g, j)', '-dfx / WX(g, i + 1) - dfy / WY(g, j)'),
 'mesh_face_area': ('-dfx / WX(g, i) - dfy / WY(g, j)', '-dfx / WY(g, j) - dfy / WX(g, i)'),
 'mesh_ghost_width': ('src = i < 0 ? -i - 1 : 2 * n - 1 - i;', 'src = i < 0 ? 0 : n - 1;'),
 'mesh_wall_distance': ('double d = 2.0 * s[k - 1];', 'double d = (2 * k - 1) * s[0] * 2.0;'),
 'mesh_wall_far_end': ('side == 1 ? WX(g, g->nx - 1 - m)', 'side == 1 ? WX(g, m)'),
 'mesh_lagrange': ('double l1 = -(s[0] + s[2]) / ((s[1] - s[0]) * (s[1] - s[2]));', 'double l1 = -(s[0] + s[2]) / ((s[1] - s[0]) * (s[2] - s[1]));'),
 'mesh_dV_swap': ('double dV = (P->xw ? P->xw[i] : P->dx) * (P->yw ? P->yw[j] : P->dx);', 'double dV = (P->xw ? P->xw[j % P->nx] : P->dx) * (P->yw ? P->yw[i % P->ny] : P->dx);'),
 'fstar_sign': ('(1.0 - 1.0 / (2.0 * tau_f)) * fneqm', '-(1.0 - 1.0 / (2.0 * tau_f)) * fneqm'),
 'kappa_sign': ('- kappa * lap', '+ kappa * lap'),
 'gamma_one': ('double Gamma = CS2 * (eu / CS2', 'double Gamma = CS2 * (1.0 + eu / CS2'),
 'drop_C_source': ('S[4] = (P->c_source == 1 ? C * (1.0 - ratio) : (1.0 - ratio)) * fs_dot;', 'S[4] = 0.0;'),
 'weight_diag': ('1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};', '1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 30.0};'),
 'FMy_ex': ('FMy += en * ey * fstar;', 'FMy += en * ex * fstar;'),
 'tauh_no_cpref': ('lam_f / (rho_f * cpref * CS2 * dt)', 'lam_f / (rho_f * CS2 * dt)'),
 'rk_coef': ('0.75 * W[q] + 0.25 * W1[q]', '0.7 * W[q] + 0.3 * W1[q]'),
 'no_projection': ('W[2 * n + q] *= (1.0 - Fs);', 'W[2 * n + q] *= 1.0;'),
 'dirichlet_ghost': ('double Tg = 2.0 * b->T_w - Tm;', 'double Tg = b->T_w;'),
 'wetting_sign': ('Wg[4] = m->W[4] + d', 'Wg[4] = m->W[4] - d'),
 'fsdot_sign': ('(solid_fraction(P, W[q], W[4 * n + q]) - Fs0[q]) / dt', '(Fs0[q] - solid_fraction(P, W[q], W[4 * n + q])) / dt'),
 'bulk_mu_factor': ('2.0 * beta * C * (C - 1.0)', 'beta * C * (C - 1.0)'),
 'side_swap': ('if (side > 0) {', 'if (side < 0) {'),
 'face_avg_one_side': ('avg[v] = 0.5 * (ra[v] + rb[v]);', 'avg[v] = ra[v];'),
 'surf_sign': ('double surf = P->surf_model == 1 ? -c->Fl * C : -C;', 'double surf = P->surf_model == 1 ? c->Fl * C : C;'),
 'surf1_sign': ('double surf = P->surf_model == 1 ? -c->Fl * C : -C;', 'double surf = P->surf_model == 1 ? c->Fl * C : -C;'),
 'surf1_solid_fraction': ('double surf = P->surf_model == 1 ? -c->Fl * C : -C;', 'double surf = P->surf_model == 1 ? -(1.0 - c->Fl) * C : -C;'),
 'surf1_as_model0': ('double surf = P->surf_model == 1 ? -c->Fl * C : -C;', 'double surf = -C;'),
 'outlet_momentum_odd': ('    } else { /* outlet: zero gradient */\n        Wg[normal] = m->W[normal];', '    } else { /* outlet: zero gradient */\n        Wg[normal] = -m->W[normal];'),
 'outlet_tangential_odd': ('    } else { /* outlet: zero gradient */\n        Wg[normal] = m->W[normal];\n        Wg[tang] = m->W[tang];', '    } else { /* outlet: zero gradient */\n        Wg[normal] = m->W[normal];\n        Wg[tang] = -m->W[tang];'),
 'outlet_no_mass_flux': ('if (b->flow != OR_FLOW_OUTLET) F[1] = 0.0;', 'F[1] = 0.0;'),
 'ibm_sign_both': [('(surf * c->grad[V_MUC][0] - c->rho * u * fs_dot', '(surf * c->grad[V_MUC][0] + c->rho * u * fs_dot'),
                   ('(surf * c->grad[V_MUC][1] - c->rho * v * fs_dot', '(surf * c->grad[V_MUC][1] + c->rho * v * fs_dot')],
 'ibm_sign': ('- c->rho * u * fs_dot', '+ c->rho * u * fs_dot'),
 'Sp_no_advect': ('S[1] = (u * drho_x + v * drho_y) * CS2 +', 'S[1] = 0.0 * (u * drho_x + v * drho_y) * CS2 +'),
 'SH_sign': ('S[0] = c->cp * c->val[V_T] * div_u;', 'S[0] = -c->cp * c->val[V_T] * div_u;'),
 'feq_quadratic': ('eu * eu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2)));\n}\n\n/* Eq. (33)', 'eu * eu / (2.0 * CS2) - uu / (2.0 * CS2)));\n}\n\n/* Eq. (33)'),
 'heq_drop_cpref': ('return w * cp * T * (cpref / cp + eu / CS2', 'return w * cp * T * (1.0 + eu / CS2'),
 'geq0_weight': ('return C - muc * Qg * (1.0 - w) / CS2;', 'return C - muc * Qg * (1.0 - 0.5 * w) / CS2;'),
 'recon_sign': ('out[v] = c->val[v] + rx * c->grad[v][0] + ry * c->grad[v][1];', 'out[v] = c->val[v] - rx * c->grad[v][0] + ry * c->grad[v][1];'),
 'recon_y_swap': ('out[v] = c->val[v] + rx * c->grad[v][0] + ry * c->grad[v][1];', 'out[v] = c->val[v] + rx * c->grad[v][0] + ry * c->grad[v][0];'),
 'point_rho_face': ('feq_pt[al] = feq(Q9_W[al], ex, ey, psi[V_P], rho_pt,', 'feq_pt[al] = feq(Q9_W[al], ex, ey, psi[V_P], rho_f,'),
 'closure_cpL': ('*T = P->T_l + (H - Hl) / cpL;', '*T = P->T_l + (H - Hl) / cpS;'),
 'mix_gas': ('(1.0 - Fs) * (1.0 - C) * g[2]', '(1.0 - C) * g[2]'),
 'wall_Fp': ('if (b->flow != OR_FLOW_OUTLET) F[1] = 0.0;', ';'),
 'gravity_y_sign': ('c->rho * P->gy);', '-c->rho * P->gy);'),
 'wall_FC': ('    F[4] = 0.0;\n    if (b->heat', '    if (b->heat'),
 'u_new_rho': ('double u_new = mx / (rho_f * CS2);', 'double u_new = mx / (CS2);'),
 'C_source_with_C': ('S[4] = (P->c_source == 1 ? C * (1.0 - ratio) : (1.0 - ratio)) * fs_dot;', 'S[4] = C * (1.0 - ratio) * fs_dot;'),
 'C_source_reading_swap': ('S[4] = (P->c_source == 1 ? C * (1.0 - ratio) : (1.0 - ratio)) * fs_dot;', 'S[4] = (P->c_source == 0 ? C * (1.0 - ratio) : (1.0 - ratio)) * fs_dot;'),
 'p_source_sign': ('c->rho * CS2 * (1.0 - ratio) * fs_dot; /* row 2 */', 'c->rho * CS2 * (ratio - 1.0) * fs_dot; /* row 2 */'),
 'p_source_no_rho': ('c->rho * CS2 * (1.0 - ratio) * fs_dot; /* row 2 */', 'CS2 * (1.0 - ratio) * fs_dot; /* row 2 */'),
 'solid_counts_gas': ('return clamp01(C) * (1.0 - Fl);', 'return (1.0 - Fl);'),
}
KEEP = ('oracle', 'tests', 'paper_2507_03366_amd')


def copy_sources(dst):
    """Copy what the pins need: the oracle source, the tests and the package's
    Python modules (never built libraries or anything else in the tree)."""
    for top in KEEP:
        for root, dirs, files in os.walk(os.path.join(SRC, top)):
            dirs[:] = [x for x in dirs if x not in ('__pycache__', '_build', 'csrc')]
            rel = os.path.relpath(root, SRC)
            os.makedirs(os.path.join(dst, rel), exist_ok=True)
            for f in files:
                if f.endswith(('.py', '.c', '.h', '.txt')):
                    shutil.copy2(os.path.join(root, f), os.path.join(dst, rel, f))


only = sys.argv[1:]
res = {}
for name, spec in MUTS.items():
    pairs = spec if isinstance(spec, list) else [spec]
    if only and name not in only: continue
    d=os.path.join(tempfile.mkdtemp(prefix='oracle_mut_'), 'repo')
    copy_sources(d)
    p=d+'/oracle/eulbfs_oracle.c'
    s=open(p).read()
    if any(a not in s for a, _ in pairs):
        res[name]='PATTERN MISSING'; print(name, res[name], flush=True); continue
    for a, b in pairs:
        s = s.replace(a, b, 1)
    open(p,'w').write(s)
    subprocess.run(['gcc','-O2','-fopenmp','-ffp-contract=off','-fPIC','-shared','-o',d+'/oracle/liboracle.so',p,'-lm'],check=True)
    r=subprocess.run([sys.executable,'-m','pytest','-q','-x','--timeout','120','tests/test_oracle_pins.py','tests/test_oracle_mesh.py','-p','no:cacheprovider'],cwd=d,capture_output=True,text=True)
    last=[l for l in r.stdout.splitlines() if 'FAILED' in l or 'passed' in l or 'failed' in l]
    res[name]='caught' if r.returncode!=0 else 'SURVIVED'
    print(name, res[name], last[:1], flush=True)
    shutil.rmtree(os.path.dirname(d), ignore_errors=True)
survived = {k: v for k, v in res.items() if v != 'caught'}
print(f"{len(res) - len(survived)} of {len(res)} mutants caught; not caught: {survived}")
sys.exit(1 if survived else 0)
