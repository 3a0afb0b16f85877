"""Mutation audit of the oracle's pins (test infrastructure; run by hand on
the CPU, not collected by pytest: about 50 minutes).

    python tests/oracle_mutation_audit.py [name-substring ...]

Copies oracle/, gen/ and tests/ into a temporary directory, plants one
plausible mistake at a time in the copy of the oracle (a dropped term, a
wrong sign, factor or index, a transposed operand, a swapped barycentric),
rebuilds the C oracle there and runs the oracle's pin tests
(tests/test_oracle_*.py, except the sanitizer build).  A mistake that no pin
catches is reported as SURVIVED.  The stored benchmark unit counts are not
run: they only check that the sources match the stored counts' hash.

Expected survivors, each a change that keeps what the pins can fix:
"no psd clamp" (B'' > 0 on (0, eps), so the clamp never acts on a face
sample), "accd mean" and "accd later step" (other shifts and step
fractions of additive CCD still give a conservative time of impact, the
property pinned against exact times), and "py armijo sign" (it only
changes which step lengths the oracle's Newton line search accepts when a
full step raises the energy, which the pinned scenes never take)."""
import os
import shutil
import subprocess
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (name, file, text, replacement, which occurrence)
MUTATIONS = [
    ('barrier sign', 'oracle/gmcp_oracle.c',
     'return -d * d * log(g / eps);',
     'return d * d * log(g / eps);', 0),
    ('barrier d1 term', 'oracle/gmcp_oracle.c',
     'return -2.0 * d * log(g / eps) - d * d / g;',
     'return -2.0 * d * log(g / eps) + d * d / g;', 0),
    ('barrier d2 coef', 'oracle/gmcp_oracle.c',
     '- 4.0 * d / g +',
     '- 2.0 * d / g +', 0),
    ('hermite cubic', 'oracle/gmcp_oracle.c',
     '3.0 * t * t - 2.0 * t * t * t',
     '3.0 * t * t - 2.0 * t * t', 0),
    ('gamma drops bm2', 'oracle/gmcp_oracle.c',
     '  if (bm[2] < mn) mn = bm[2];\n  return ora_hermite',
     '  return ora_hermite', 0),
    ('rest area half', 'oracle/gmcp_oracle.c',
     'area[t] = 0.5 * v_norm(n);',
     'area[t] = v_norm(n);', 0),
    ('ray bary swap', 'oracle/gmcp_oracle.c',
     '  bm[1] = b1;\n  bm[2] = b2;\n  *t_out',
     '  bm[1] = b2;\n  bm[2] = b1;\n  *t_out', 0),
    ('ray b1 coef', 'oracle/gmcp_oracle.c',
     'double b1 = (a22 * r1 - a12 * r2) / det;\n  double b2',
     'double b1 = (a11 * r1 - a12 * r2) / det;\n  double b2', 0),
    ('narrow farthest', 'oracle/gmcp_oracle.c',
     'if (best < 0 || t < bt || (t == bt && M < best))',
     'if (best < 0 || t > bt || (t == bt && M < best))', 0),
    ('narrow facing flip', 'oracle/gmcp_oracle.c',
     'if (den >= 0.0) continue; /* not opposing */',
     'if (den <= 0.0) continue; /* not opposing */', 0),
    ('narrow outside kept', 'oracle/gmcp_oracle.c',
     'if (mb < 0.0) continue; /* outside */',
     'if (mb < -0.05) continue; /* outside */', 0),
    ('weight factor 2', 'oracle/gmcp_oracle.c',
     'double w = 2.0 * area[T] * rule[3 * q + 2];',
     'double w = area[T] * rule[3 * q + 2];', 0),
    ('c2 drops gamma', 'oracle/gmcp_oracle.c',
     'c2[k] = kappa * w * gam * B2;',
     'c2[k] = kappa * w * B2;', 0),
    ('grad slave sign', 'oracle/gmcp_oracle.c',
     '+= -c1[k] * bs[a] * n[d];',
     '+= c1[k] * bs[a] * n[d];', 0),
    ('grad master bary index', 'oracle/gmcp_oracle.c',
     '+= c1[k] * bmv[3 * k + j] * n[d];',
     '+= c1[k] * bmv[3 * k + (j + 1) % 3] * n[d];', 0),
    ('hess slave bary swap', 'oracle/gmcp_oracle.c',
     'double s[6] = {-(1.0 - xi - eta), -xi, -eta,',
     'double s[6] = {-(1.0 - xi - eta), -eta, -xi,', 0),
    ('hess coef transposed', 'oracle/gmcp_oracle.c',
     'double coef = c2[k] * s[hc[i].a] * s[hc[i].b];',
     'double coef = c2[k] * s[hc[i].a] * s[hc[i].a];', 0),
    ('no psd clamp', 'oracle/gmcp_oracle.c',
     '} else if (c2[k] < 0.0) {',
     '} else if (0) {', 0),
    ('pressure drops gamma', 'oracle/gmcp_oracle.c',
     'if (press) press[k] = -kappa * gam * B1;',
     'if (press) press[k] = -kappa * B1;', 0),
    ('assemble eps from gref', 'oracle/gmcp_oracle.c',
     'if (g_ref && 0.9 * g_ref[k] < eps) eps = 0.9 * g_ref[k];',
     'if (g_ref && 0.9 * g_ref[k] < eps) eps = g_ref[k];', 1),
    ('linear bound 0.9', 'oracle/gmcp_oracle.c',
     'double a = 0.9 * g / (-gd);',
     'double a = g / (-gd);', 0),
    ('linear bound master sign', 'oracle/gmcp_oracle.c',
     'gd += bm[j] * v_dot(n, dxm',
     'gd -= bm[j] * v_dot(n, dxm', 0),
    ('ptri inside test', 'oracle/gmcp_oracle.c',
     'if (b1 >= 0.0 && b2 >= 0.0 && b1 + b2 <= 1.0) return s * s * nn;',
     'if (b1 >= 0.0 && b2 >= 0.0) return s * s * nn;', 0),
    ('ptri edge dropped', 'oracle/gmcp_oracle.c',
     '  if (d3 < d) d = d3;\n  return d;',
     '  return d;', 0),
    ('accd mean', 'oracle/gmcp_oracle.c',
     'mean[d] = 0.25 * (dp[d] + da[d] + db[d] + dc[d]);',
     'mean[d] = 0.25 * (da[d] + db[d] + dc[d]);', 0),
    ('accd bound l', 'oracle/gmcp_oracle.c',
     'double l = v_norm(u[0]) + lt;',
     'double l = lt;', 0),
    ('accd later step', 'oracle/gmcp_oracle.c',
     'step = 0.9 * dist / l;',
     'step = dist / l;', 0),
    ('swept box dx', 'oracle/gmcp_oracle.c',
     'double v0 = v[d], v1 = v[d] + (dxm ? dxm[3 * (int64_t)tm[3 * t + j] + d] : 0.0);',
     'double v0 = v[d], v1 = v[d];', 0),
    ('py clip intersection', 'oracle/mortar.py',
     'out.append(P + (Q - P) * (fp / (fp - fq)))',
     'out.append(P + (Q - P) * (fq / (fp - fq)))', 0),
    ('py clip boundary', 'oracle/mortar.py',
     '            if fp >= 0.0:',
     '            if fp > 0.0:', 0),
    ('py mortar weight 2', 'oracle/mortar.py',
     '2.0 * (a2 * area_rest) * wq',
     '(a2 * area_rest) * wq', 0),
    ('py mortar bm swap', 'oracle/mortar.py',
     'bm = np.array([1.0 - b12[0] - b12[1], b12[0], b12[1]])',
     'bm = np.array([1.0 - b12[0] - b12[1], b12[1], b12[0]])', 0),
    ('py mortar facing', 'oracle/mortar.py',
     'if n @ np.cross(m[1] - m[0], m[2] - m[0]) >= 0.0:',
     'if n @ np.cross(m[1] - m[0], m[2] - m[0]) <= 0.0:', 0),
    ('py mortar fan last', 'oracle/mortar.py',
     'for i in range(1, len(poly) - 1):',
     'for i in range(1, len(poly) - 2):', 0),
    ('py mortar gap sign', 'oracle/mortar.py',
     'g = float(n @ (bm @ m - xs_k))',
     'g = float(n @ (xs_k - bm @ m))', 0),
    ('py edge gamma', 'oracle/mortar.py',
     '(oracle.hermite(smp.eta, delta_e) * oracle.hermite(1.0 - smp.eta, delta_e))',
     'oracle.hermite(smp.eta, delta_e)', 0),
    ('py lame mu', 'oracle/fem.py',
     'mu = young / (2.0 * (1.0 + poisson))',
     'mu = young / (1.0 + poisson)', 0),
    ('py stiffness transposed', 'oracle/fem.py',
     '+ mu * np.einsum("ni,nk->nik", g[:, b], g[:, a])',
     '+ mu * np.einsum("ni,nk->nik", g[:, a], g[:, b])', 0),
    ('py tet volume', 'oracle/fem.py',
     'vol = np.abs(np.linalg.det(Dm)) / 6.0',
     'vol = np.abs(np.linalg.det(Dm)) / 3.0', 0),
    ('py energy lambda half', 'oracle/fem.py',
     '+ 0.5 * lam * tr * tr',
     '+ lam * tr * tr', 0),
    ('py silu grad', 'oracle/mlp.py',
     'return s * (1.0 + z * (1.0 - s))',
     'return s * (1.0 + z * s)', 0),
    ('py backward W3 input', 'oracle/mlp.py',
     'g["W3"] = H2.T @ dZ3',
     'g["W3"] = H3.T @ dZ3', 0),
    ('py mse factor', 'oracle/mlp.py',
     '2.0 * d / (B * n_out)',
     'd / (B * n_out)', 0),
    ('py adam bias corr', 'oracle/mlp.py',
     'vh = v / (1 - b2 ** step)',
     'vh = v', 0),
    ('py dual offset', 'oracle/dualmesh.py',
     '+ D[i] * n',
     '', 0),
    ('py dual bary order', 'oracle/dualmesh.py',
     'return 1.0 - v - w, v, w, float(d @ n)',
     'return 1.0 - v - w, w, v, float(d @ n)', 0),
    ('py stroud eta', 'oracle/rule.py',
     'out[q, 1] = v[j] * (1.0 - u[i])',
     'out[q, 1] = v[j]', 0),
    ('py stroud weight', 'oracle/rule.py',
     'wu = wj / 4.0',
     'wu = wj / 2.0', 0),
    ('ploss dp drops gamma', 'oracle/gmcp_oracle.c',
     'dp = -kappa * gam * ora_barrier_d2(g, eps);',
     'dp = -kappa * ora_barrier_d2(g, eps);', 0),
    ('ploss slave sign', 'oracle/gmcp_oracle.c',
     '+= r * dp * (-bs[a]) * n[d];',
     '+= r * dp * (bs[a]) * n[d];', 0),
    ('ploss ddelta', 'oracle/gmcp_oracle.c',
     'dLddelta[k] = act ? r * dp : 0.0;',
     'dLddelta[k] = act ? r : 0.0;', 0),
    ('hvp master index', 'oracle/gmcp_oracle.c',
     'dot += bm[j] * v_dot(n, vx + 3 * ((int64_t)Vs + tm[3 * M[k] + j]));',
     'dot += bm[j] * v_dot(n, vx + 3 * ((int64_t)Vs + tm[3 * M[k] + (j + 1) % 3]));', 0),
    ('hvp vd dropped', 'oracle/gmcp_oracle.c',
     '    if (vd) dot += vd[k];\n',
     '', 0),
    ('hvp slave sign', 'oracle/gmcp_oracle.c',
     'out_x[3 * (int64_t)ts[3 * T + a] + d] += s * (-bs[a]) * n[d];',
     'out_x[3 * (int64_t)ts[3 * T + a] + d] += s * (bs[a]) * n[d];', 0),
    ('swept count pad', 'oracle/gmcp_oracle.c',
     'lo[d] = l - (pad_rel * fabs(l) + pad_abs);',
     'lo[d] = l;', 0),
    ('swept count end', 'oracle/gmcp_oracle.c',
     'double e = p + (b0 * dA[d] + xi * dB[d] + eta * dC[d]);',
     'double e = p + (b0 * dA[d] + xi * dB[d] + xi * dC[d]);', 0),
    ('ccd swept dp', 'oracle/gmcp_oracle.c',
     'dp[d] = b0 * dA[d] + xi * dB[d] + eta * dC[d];',
     'dp[d] = b0 * dA[d] + xi * dB[d];', 0),
    ('sample geom point', 'oracle/gmcp_oracle.c',
     'p[d] = s0[d] + rule[3 * q] * e1[d] + rule[3 * q + 1] * e2[d];',
     'p[d] = s0[d] + rule[3 * q + 1] * e1[d] + rule[3 * q] * e2[d];', 0),
    ('slave normal orientation', 'oracle/gmcp_oracle.c',
     'v_cross(e1, e2, cr);',
     'v_cross(e2, e1, cr);', 0),
    ('py edge weight length', 'oracle/mortar.py',
     'L * (t1 - t0) * wj',
     '(t1 - t0) * wj', 0),
    ('py edge gap', 'oracle/mortar.py',
     'float((1.0 - eta) * ha + eta * hb)',
     'float(eta * ha + (1.0 - eta) * hb)', 0),
    ('py point strictly inside', 'oracle/mortar.py',
     'if y[0] > 0.0 and y[1] > 0.0 and 1.0 - y[0] - y[1] > 0.0:',
     'if y[0] > 0.0 and y[1] > 0.0:', 0),
    ('py mortar linear 0.9', 'oracle/mortar.py',
     'a = min(a, 0.9 * s.g / (-gd))',
     'a = min(a, s.g / (-gd))', 0),
    ('py mortar linear master', 'oracle/mortar.py',
     'gd += s.n @ (s.bm @ dxm[s.mv])',
     'gd -= s.n @ (s.bm @ dxm[s.mv])', 0),
    ('py weights factor', 'oracle/__init__.py',
     'return (2.0 * area[:, None] * P.rule[None, :, 2]).ravel()',
     'return (area[:, None] * P.rule[None, :, 2]).ravel()', 0),
    ('py mass quarter', 'oracle/fem.py',
     'rho * vol / 4.0',
     'rho * vol / 3.0', 0),
    ('py inertia dt2', 'oracle/fem.py',
     'g = (self.m[:, None] * dv / dt2).ravel() + Ku',
     'g = (self.m[:, None] * dv / self.dt).ravel() + Ku', 0),
    ('py stress mu', 'oracle/fem.py',
     '+ 2.0 * mu * eps',
     '+ mu * eps', 0),
    ('grid cell range', 'oracle/gmcp_oracle.c',
     'c1[d] = clampi((int64_t)floor((hi[d] - g->lo[d]) / g->h), 0, g->nc[d] - 1);',
     'c1[d] = clampi((int64_t)floor((hi[d] - g->lo[d]) / g->h) - 1, 0, g->nc[d] - 1);', 0),
    ('grid box test', 'oracle/gmcp_oracle.c',
     'if (a[0] > hi[0] || b[0] < lo[0] || a[1] > hi[1] || b[1] < lo[1] || a[2] > hi[2] || b[2] < lo[2])\n            continue;\n          if (cnt < cap)',
     'if (a[0] > hi[0] || b[0] < lo[0] || a[1] > hi[1] || b[1] < lo[1])\n            continue;\n          if (cnt < cap)', 0),
    ('py newton bound ignored', 'oracle/fem.py',
     'alpha = min(1.0, step_bound(P, nr, A, d))',
     'alpha = 1.0', 0),
    ('py armijo sign', 'oracle/fem.py',
     'if En <= E0 + armijo * alpha * slope or',
     'if En <= E0 - armijo * alpha * slope or', 0),
    ('py mlp skip activation', 'oracle/mlp.py',
     'Z2 = H1 @ w["W2"] + w["b2"]',
     'Z2 = Z1 @ w["W2"] + w["b2"]', 0),
    ('py adam m', 'oracle/mlp.py',
     'm = b1 * m + (1 - b1) * g',
     'm = b1 * m + g', 0),
    ('py weights rest areas', 'oracle/__init__.py',
     'area = rest_area(P.xs_rest, P.ts)\n    return (2.0',
     'area = rest_area(P.xs, P.ts)\n    return (2.0', 0),
    ('py assemble rest areas', 'oracle/__init__.py',
     '    area = rest_area(P.xs_rest, P.ts)\n    Ek, c1, c2, pr',
     '    area = rest_area(P.xs, P.ts)\n    Ek, c1, c2, pr', 0),
    ('py mortar rest areas', 'oracle/mortar.py',
     'area = oracle.rest_area(P.xs_rest, P.ts)',
     'area = oracle.rest_area(P.xs, P.ts)', 0),
    ('py dual edge clip', 'oracle/dualmesh.py',
     't = np.clip(((p - s0) * e).sum(1) / (e * e).sum(1), 0.0, 1.0)',
     't = ((p - s0) * e).sum(1) / (e * e).sum(1)', 0),
    ('py edge gauss weights', 'oracle/mortar.py',
     'xg, wg = (xg + 1.0) / 2.0, wg / 2.0',
     'xg, wg = (xg + 1.0) / 2.0, wg', 0),
]


def _copy(dst):
    for d in ("oracle", "gen", "tests"):
        shutil.copytree(os.path.join(ROOT, d), os.path.join(dst, d),
                        ignore=shutil.ignore_patterns("__pycache__", "*.so", "golden"))
    shutil.copy(os.path.join(ROOT, "pytest.ini"), dst)


def _run(work):
    b = subprocess.run([sys.executable, "-m", "oracle.build"], cwd=work, capture_output=True, text=True)
    if b.returncode:
        return True, "the oracle does not build"
    tests = sorted(os.path.join("tests", f) for f in os.listdir(os.path.join(work, "tests"))
                   if f.startswith("test_oracle_") and f.endswith(".py") and f != "test_oracle_sanitize.py")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu", "-p", "no:cacheprovider",
                        *tests], cwd=work, capture_output=True, text=True)
    tail = [ln for ln in r.stdout.splitlines() if ln.strip()][-1:]
    return r.returncode != 0, tail[0] if tail else ""


def main(only):
    with tempfile.TemporaryDirectory(prefix="oracle_mutation_") as work:
        _copy(work)
        failed, tail = _run(work)
        print("unmutated:", "FAILS " if failed else "passes", tail, flush=True)
        if failed:
            return
        for name, path, old, new, occ in MUTATIONS:
            if only and not any(o in name for o in only):
                continue
            p = os.path.join(work, path)
            with open(p) as fh:
                src = fh.read()
            parts = src.split(old)
            if len(parts) < occ + 2:
                print(f"{name}: text not found", flush=True)
                continue
            with open(p, "w") as fh:
                fh.write(old.join(parts[:occ + 1]) + new + old.join(parts[occ + 1:]))
            failed, tail = _run(work)
            print(f"{name}: {'KILLED' if failed else 'SURVIVED'} ({tail})", flush=True)
            with open(p, "w") as fh:
                fh.write(src)


if __name__ == "__main__":
    main(sys.argv[1:])
