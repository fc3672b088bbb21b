"""Planted mistakes: each entry below changes one expression of the oracle's C
source (a plausible slip: a sign, an index, a factor, a transposed operand);
every one is compiled into a scratch copy of the oracle, in a temporary
directory, and the CPU pins are run against it.  A pin set that lets a mistake
through has a gap.  The committed oracle is never modified.

Usage: python tests/oracle_mutants.py [index ...]   (a few minutes on 4 workers)
"""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import tempfile

R = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = open(os.path.join(R, "oracle", "mclbm_oracle.c")).read()
MUT = [
 ("axis weight", "{4.0 / 9.0, 1.0 / 9.0,", "{4.0 / 9.0, 1.0 / 8.0,"),
 ("opposite of diagonals", "{0, 3, 4, 1, 2, 7, 8, 5, 6}", "{0, 3, 4, 1, 2, 8, 7, 6, 5}"),
 ("feq second-moment factor", "out[q] = W[q] * (r + cj / cs2 + contr / (2.0 * cs2 * cs2));", "out[q] = W[q] * (r + cj / cs2 + contr / (4.0 * cs2 * cs2));"),
 ("feq shear term", "2.0 * Axy * (cx * cy)", "Axy * (cx * cy)"),
 ("feq momentum sign", "out[q] = W[q] * (r + cj / cs2 +", "out[q] = W[q] * (r - cj / cs2 +"),
 ("psi factor", "out[q] = W[q] * (cq[q][0] * S[0] + cq[q][1] * S[1]) / cs2;", "out[q] = W[q] * (cq[q][0] * S[0] + cq[q][1] * S[1]) / (2.0 * cs2);"),
 ("forcing factor dropped", "out[q] = f[q] - omega * (f[q] - feq[q]) + (1.0 - 0.5 * omega) * psi[q] * dt;", "out[q] = f[q] - omega * (f[q] - feq[q]) + psi[q] * dt;"),
 ("collision j without half source", "double jj[2] = {mx + 0.5 * dt * S[0], my + 0.5 * dt * S[1]};", "double jj[2] = {mx, my};"),
 ("relaxation sign", "out[q] = f[q] - omega * (f[q] - feq[q])", "out[q] = f[q] + omega * (f[q] - feq[q])"),
 ("plane stress lambda", "return 2.0 * mu * nu / (1.0 - 2.0 * nu);", "return 2.0 * mu * nu / (1.0 - nu);"),
 ("SVK E quadratic term", "E[a][b] = 0.5 * (Hm[b][a] + Hm[a][b] + HtH);", "E[a][b] = 0.5 * (Hm[b][a] + Hm[a][b]) + HtH;"),
 ("SVK H H^T for H^T H", "double HtH = Hm[0][a] * Hm[0][b] + Hm[1][a] * Hm[1][b];\n                E[a][b]", "double HtH = Hm[a][0] * Hm[b][0] + Hm[a][1] * Hm[b][1];\n                E[a][b]"),
 ("SVK lambda tr E", "S2[a][b] = (a == b ? lam * trE : 0.0) + 2.0 * mu * E[a][b];", "S2[a][b] = (a == b ? lam * trE : 0.0) + mu * E[a][b];"),
 ("NH J^2-1", "double J2m1 = Jm1 * (Jm1 + 2.0);", "double J2m1 = Jm1 * (Jm1 + 1.0);"),
 ("NH inverse sign", "{{C[1][1] / detC, -C[0][1] / detC},", "{{C[1][1] / detC, C[0][1] / detC},"),
 ("NH det H dropped", "double Jm1 = (Hm[0][0] + Hm[1][1]) + (Hm[0][0] * Hm[1][1] - Hm[0][1] * Hm[1][0]);", "double Jm1 = (Hm[0][0] + Hm[1][1]);"),
 ("P = S F instead of F S", "P[2 * a + b] = F[a][0] * S2[0][b] + F[a][1] * S2[1][b];", "P[2 * a + b] = S2[a][0] * F[0][b] + S2[a][1] * F[1][b];"),
 ("linear law lambda", "P[2 * a + b] = (a == b ? lam * tr : 0.0) + mu * (Hm[a][b] + Hm[b][a]);", "P[2 * a + b] = (a == b ? mu * tr : 0.0) + mu * (Hm[a][b] + Hm[b][a]);"),
 ("Pi(H) shear index", "Pi[1] = -(mu * (H[1] + H[2]));", "Pi[1] = -(mu * (H[1] + H[1]));"),
 ("Pi(H) trace sign", "Pi[0] = -(mu * (H[0] + H[0]) + mu * tr);", "Pi[0] = -(mu * (H[0] + H[0]) - mu * tr);"),
 ("cs2 = mu / (3 rho0)", "h->cs2 = mu / rho0;", "h->cs2 = mu / rho0 / 3.0;"),
 ("dt halved", "h->dt = dx / h->c;", "h->dt = 0.5 * dx / h->c;"),
 ("one-sided sign", "return s * (AT(1) - AT(0)) / h->dx;", "return (AT(1) - AT(0)) / h->dx;"),
 ("one-sided over 2 dX", "return s * (AT(1) - AT(0)) / h->dx;", "return s * (AT(1) - AT(0)) / (2.0 * h->dx);"),
 ("central difference over dX", "mp = m + 1; mm = m - 1; div = 2.0 * h->dx;", "mp = m + 1; mm = m - 1; div = h->dx;"),
 ("periodic wrap off by one", "mp = (m + 1) % L; mm = (m - 1 + L) % L;", "mp = (m + 1) % L; mm = (m - 2 + L) % L;"),
 ("Div of T^T", "S[i] = h->rho0 * h->body[0] + (fd(h, T + 0 * N, x, y, 0) + fd(h, T + 1 * N, x, y, 1));", "S[i] = h->rho0 * h->body[0] + (fd(h, T + 0 * N, x, y, 0) + fd(h, T + 2 * N, x, y, 1));"),
 ("body force sign", "S[i] = h->rho0 * h->body[0] +", "S[i] = -h->rho0 * h->body[0] +"),
 ("init r0 sign", "double r0 = -h->rho0 * (H[0] + H[3]);", "double r0 = h->rho0 * (H[0] + H[3]);"),
 ("Neumann normal traction sign", "double Paa = -s * Ts[a] + EXT(T_aa);", "double Paa = s * Ts[a] + EXT(T_aa);"),
 ("Neumann shear from T_aa", "double Pab = -s * Ts[b] + EXT(T_ba);", "double Pab = -s * Ts[b] + EXT(T_aa);"),
 ("Neumann Pi_bb zero", "double Pbb = EXT(Pi_bb);", "double Pbb = 0.0;"),
 ("Neumann Pi_bb wrong plane", "(b == 0 ? 0 : 2)", "(b == 0 ? 2 : 0)"),
 ("corner shear one wall", "PiC[1] = 0.5 * (PiX[1] + PiY[1]);", "PiC[1] = PiX[1];"),
 ("bounce-back sign", "val = fcq - 2.0 / cs2 * W[q] * (cqx * js[0] + cqy * js[1]);", "val = fcq + 2.0 / cs2 * W[q] * (cqx * js[0] + cqy * js[1]);"),
 ("anti-bounce-back sign", "val = -fcq + 2.0 * W[q] * (r + contr / (2.0 * cs2 * cs2));", "val = fcq + 2.0 * W[q] * (r + contr / (2.0 * cs2 * cs2));"),
 ("anti-bounce-back without r", "val = -fcq + 2.0 * W[q] * (r + contr / (2.0 * cs2 * cs2));", "val = -fcq + 2.0 * W[q] * (contr / (2.0 * cs2 * cs2));"),
 ("forward Euler update", "h->un[i] = h->u[i] + dt / (2.0 * h->rho0) * (jx + h->jA[i]);", "h->un[i] = h->u[i] + dt / h->rho0 * jx;"),
 ("update j without half source", "double jx = mx + 0.5 * dt * S[i],", "double jx = mx,"),
 ("ramp off by one", "double k = (double)n < s->t1 ?", "double k = (double)n <= s->t1 ?"),
 ("gauss width", "return exp(-d * d / (2.0 * s->width * s->width));", "return exp(-d * d / (s->width * s->width));"),
 ("sin2 ramp period", "double v = sin(M_PI * n / (2.0 * s->t1));", "double v = sin(M_PI * n / s->t1);"),
 ("push instead of pull", "int xt = x + EX[q], yt = y + EY[q];\n                if (px)", "int xt = x - EX[q], yt = y - EY[q];\n                if (px)"),
 ("TRT even/odd swapped", "double even = 0.5 * (nq + nb), odd = 0.5 * (nq - nb);", "double even = 0.5 * (nq - nb), odd = 0.5 * (nq + nb);"),
 ("linear extrapolation sign", "0.5 * (3.0 * (arr)[i] - (arr)[ii])", "0.5 * (3.0 * (arr)[i] + (arr)[ii])"),
 ("second-order one-sided coefficient", "s * (-3.0 * AT(0) + 4.0 * AT(1) - AT(2))", "s * (-3.0 * AT(0) + 4.0 * AT(1) + AT(2))"),
 ("cq y from EX", "h->cq[q][1] = h->c * EY[q];", "h->cq[q][1] = h->c * EX[q];"),
 ("one diagonal weight", "1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0}", "1.0 / 36.0, 1.0 / 32.0, 1.0 / 36.0, 1.0 / 36.0}"),
 ("one velocity sign", "static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};", "static const int EY[9] = {0, 0, 1, 0, -1, 1, -1, -1, -1};"),
 ("feq r term sign", "double Axx = Pi[0] - r * cs2, Axy = Pi[1], Ayy = Pi[2] - r * cs2;", "double Axx = Pi[0] + r * cs2, Axy = Pi[1], Ayy = Pi[2] + r * cs2;"),
 ("psi transposed", "out[q] = W[q] * (cq[q][0] * S[0] + cq[q][1] * S[1]) / cs2;", "out[q] = W[q] * (cq[q][1] * S[0] + cq[q][0] * S[1]) / cs2;"),
 ("collision Pi_xy moment", "        pxy += cq[q][0] * cq[q][1] * f[q];\n        pyy += cq[q][1] * cq[q][1] * f[q];\n    }\n    double jj[2] = {mx + 0.5 * dt * S[0], my + 0.5 * dt * S[1]};\n    double Pi3[3] = {pxx, pxy, pyy};\n    double feq[9], psi[9];\n    orc_feq(cs2, cq, r, jj, Pi3, feq);\n    orc_psi(cs2, cq, S, psi);\n    for (int q = 0; q < 9; q++)\n        out[q] = f[q] - omega", "        pxy += cq[q][0] * cq[q][0] * f[q];\n        pyy += cq[q][1] * cq[q][1] * f[q];\n    }\n    double jj[2] = {mx + 0.5 * dt * S[0], my + 0.5 * dt * S[1]};\n    double Pi3[3] = {pxx, pxy, pyy};\n    double feq[9], psi[9];\n    orc_feq(cs2, cq, r, jj, Pi3, feq);\n    orc_psi(cs2, cq, S, psi);\n    for (int q = 0; q < 9; q++)\n        out[q] = f[q] - omega"),
 ("TRT forcing at the even rate", "out[q] = f[q] - omega_plus * even - omega * odd + (1.0 - 0.5 * omega) * psi[q] * dt;", "out[q] = f[q] - omega_plus * even - omega * odd + (1.0 - 0.5 * omega_plus) * psi[q] * dt;"),
 ("Pi(H) yy from H_xx", "Pi[3] = -(mu * (H[3] + H[3]) + mu * tr);", "Pi[3] = -(mu * (H[0] + H[0]) + mu * tr);"),
 ("NH det C sign", "double detC = C[0][0] * C[1][1] - C[0][1] * C[1][0];", "double detC = C[0][0] * C[1][1] + C[0][1] * C[1][0];"),
 ("source y axes swapped", "(fd(h, T + 2 * N, x, y, 0) + fd(h, T + 3 * N, x, y, 1));", "(fd(h, T + 2 * N, x, y, 1) + fd(h, T + 3 * N, x, y, 0));"),
 ("inward neighbour outward", "int xi = x - (a == 0 ? (int)s : 0), yi = y - (a == 1 ? (int)s : 0);", "int xi = x + (a == 0 ? (int)s : 0), yi = y + (a == 1 ? (int)s : 0);"),
 ("traction at the next step", "    side_value(h, side, n, Ts);", "    side_value(h, side, n + 1, Ts);"),
 ("wall momentum at the next step", "double v[2]; side_value(h, wx, n, v);", "double v[2]; side_value(h, wx, n + 1, v);"),
 ("corner j* not averaged", "js[0] /= nd; js[1] /= nd;", "js[0] /= 1; js[1] /= 1;"),
 ("initial j_y from j_x", "double jj[2] = {j0 ? j0[i] : 0.0, j0 ? j0[N + i] : 0.0};", "double jj[2] = {j0 ? j0[i] : 0.0, j0 ? j0[i] : 0.0};"),
 ("periodic x wrap shifted", "if (px) xt = (xt + nx) % nx;", "if (px) xt = (xt + nx + 1) % nx;"),
 ("linear ramp one step late", "case LOAD_LINEAR_RAMP: return n < s->t1 ? n / s->t1 : 1.0;", "case LOAD_LINEAR_RAMP: return n < s->t1 ? (n + 1) / s->t1 : 1.0;"),
 ("sin pulse period", "case LOAD_SIN_PULSE: return n < s->t1 ? sin(M_PI * n / s->t1) : 0.0;", "case LOAD_SIN_PULSE: return n < s->t1 ? sin(2.0 * M_PI * n / s->t1) : 0.0;"),
 ("Ricker amplitude", "double a = 2.0 / sqrt(3.0 * s->width * sqrt(M_PI));", "double a = 1.0 / sqrt(3.0 * s->width * sqrt(M_PI));"),
 ("update without rho0", "h->un[i] = h->u[i] + dt / (2.0 * h->rho0) * (jx + h->jA[i]);", "h->un[i] = h->u[i] + dt / 2.0 * (jx + h->jA[i]);"),
 ("trapezoid uses new j twice", "h->un[N + i] = h->u[N + i] + dt / (2.0 * h->rho0) * (jy + h->jA[N + i]);", "h->un[N + i] = h->u[N + i] + dt / (2.0 * h->rho0) * (jy + jy);"),
 ("diag kinetic energy without the half", "ek += (jx * jx + jy * jy) / (2.0 * h->rho0);", "ek += (jx * jx + jy * jy) / h->rho0;"),
 ("diag max |u| squared", "out[3] = sqrt(mu2);", "out[3] = mu2;"),
 ("diag flag ignores j", "if (!isfinite(jx) || !isfinite(jy) || !isfinite(ux)", "if (!isfinite(ux)"),
 ("diag momentum y from j_x", "sx += jx; sy += jy;", "sx += jx; sy += jx;"),
 ("diag |u| from u_x only", "double m = ux * ux + uy * uy;", "double m = ux * ux;"),
 ("corner options swapped", "h->corner == 1 ? PiX[1] : (h->corner == 2 ? PiY[1]", "h->corner == 1 ? PiY[1] : (h->corner == 2 ? PiX[1]"),
 ("table one step ahead", "return s->table[k < s->table_len ? k : s->table_len - 1];", "return s->table[k + 1 < s->table_len ? k + 1 : s->table_len - 1];"),
]
TESTS = ["tests/test_oracle_blocks.py", "tests/test_oracle_invariants.py", "tests/test_paper_cases.py"]

def one(k):
    name, old, new = MUT[k]
    assert SRC.count(old) >= 1, name
    d = tempfile.mkdtemp(prefix=f"oracle_mutant{k:02d}_")
    os.makedirs(os.path.join(d, "oracle"))
    shutil.copytree(os.path.join(R, "tests"), os.path.join(d, "tests"), ignore=shutil.ignore_patterns("__pycache__"))
    os.symlink(os.path.join(R, "paper_2502_00920_amd"), os.path.join(d, "paper_2502_00920_amd"))
    shutil.copy(os.path.join(R, "oracle", "__init__.py"), os.path.join(d, "oracle"))
    open(os.path.join(d, "oracle", "mclbm_oracle.c"), "w").write(SRC.replace(old, new, 1))
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
                           "-o", os.path.join(d, "oracle", "liboracle.so"), os.path.join(d, "oracle", "mclbm_oracle.c"), "-lm"])
    env = dict(os.environ, OMP_NUM_THREADS="2")
    p = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu", "-p", "no:cacheprovider", *TESTS],
                       cwd=d, capture_output=True, text=True, env=env, timeout=900)
    failed = [l for l in p.stdout.splitlines() if l.startswith("FAILED") or l.startswith("ERROR")]
    shutil.rmtree(d, ignore_errors=True)
    return k, name, p.returncode, failed[:1]

if __name__ == "__main__":
    ks = range(len(MUT)) if len(sys.argv) == 1 else [int(a) for a in sys.argv[1:]]
    survived = 0
    with cf.ThreadPoolExecutor(4) as ex:
        for k, name, rc, failed in ex.map(one, ks):
            survived += rc == 0
            print(f"{k:2d} {'caught  ' if rc != 0 else 'SURVIVED'} {name:38s} {failed[0][:110] if failed else ''}",
                  flush=True)
    print(f"{survived} of {len(ks)} planted mistakes passed every pin")
    sys.exit(1 if survived else 0)
