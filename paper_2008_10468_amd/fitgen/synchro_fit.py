"""Offline generator of the piecewise fits of the synchrotron functions used by the
GPU kernels (writes ``csrc/synchro_coeffs.inc``).

Representation (shared by FP32 and FP64 tables).  With t = x^(1/3),

    F(x) = t e^{-x} H_F(t),    G(x) = t e^{-x} H_G(t),

where F(x) = x int_x^inf K_{5/3} and G(x) = x K_{2/3} (Sec. 3.2.1).  The small-x
series of Sec. 3.2.1 shows that F/x^(1/3) and G/x^(1/3) are power series in
x^(1/3) (they contain x^0, x^(2/3), x^(4/3), x^2, ... only), so H_F and H_G are
analytic in t on [0, inf), bounded near 0 (H_F(0) = 2^(2/3) Gamma(2/3),
H_G(0) = 2^(-1/3) Gamma(2/3)) and grow like sqrt(pi/2) t^(1/2) at large t (the
large-x form L(x) of Sec. 3.2.1).  Unlike the paper's medium-range form
x^(1/3) M - x^(5/3) P, nothing cancels, so one formula holds on the whole range
and the segment is picked arithmetically from t (no branches per range).

Each segment [t_j, t_j + w] holds a polynomial in s = (t - c_j)/(w/2) in [-1, 1],
obtained by Chebyshev interpolation on first-kind nodes (near-minimax) and
converted to monomial coefficients in 50-digit arithmetic before rounding to the
table's precision.

Reference values: the integral representations
    F(x) = x e^{-x} int_0^inf e^{-2x sinh^2(t/2)} cosh(5t/3)/cosh t dt,
    G(x) = x e^{-x} int_0^inf e^{-2x sinh^2(t/2)} cosh(2t/3) dt
evaluated with mpmath's tanh-sinh quadrature at 40 digits, split at multiples of
the peak width.  Run: ``python -m paper_2008_10468_amd.fitgen.synchro_fit``.
"""
from __future__ import annotations

import multiprocessing as mpc
import os
import sys

import mpmath as mp

# Table layouts: (name, ctype, segment width in t, number of segments, degree)
TABLES = (
    ("f32", "float", mp.mpf(1) / 2, 9, 7),     # t in [0, 4.5]:  x <= 91.1
    ("f64", "double", mp.mpf(1) / 4, 37, 11),  # t in [0, 9.25]: x <= 791
)

DPS = 40


def _H(t):
    """(H_F(t), H_G(t)) at high precision."""
    mp.mp.dps = DPS
    t = mp.mpf(t)
    if t == 0:
        g23 = mp.gamma(mp.mpf(2) / 3)
        return (mp.mpf(2) ** (mp.mpf(2) / 3) * g23, mp.mpf(2) ** (-mp.mpf(1) / 3) * g23)
    x = t ** 3
    c53 = mp.mpf(5) / 3
    c23 = mp.mpf(2) / 3
    top = mp.acosh(1 + (100 + mp.log(1 + 1 / x)) / x) + 1
    width = min(mp.mpf(1) / 2, 1 / mp.sqrt(x))
    pts = [mp.mpf(0)]
    while pts[-1] < top:
        pts.append(pts[-1] + width)
    i1 = mp.quad(lambda s: mp.exp(-2 * x * mp.sinh(s / 2) ** 2) * mp.cosh(c53 * s) / mp.cosh(s), pts)
    i2 = mp.quad(lambda s: mp.exp(-2 * x * mp.sinh(s / 2) ** 2) * mp.cosh(c23 * s), pts)
    # F = x e^{-x} I1 = t e^{-x} (t^2 I1)
    return (t * t * i1, t * t * i2)


def _cheb_to_monomial(vals, d):
    """Chebyshev interpolant on first-kind nodes -> monomial coefficients in s."""
    n = d + 1
    a = []
    for k in range(n):
        s = mp.mpf(0)
        for j in range(n):
            s += vals[j] * mp.cos(mp.pi * k * (j + mp.mpf(1) / 2) / n)
        a.append(2 * s / n)
    a[0] /= 2
    # T_k(s) in monomials by the three-term recurrence
    T = [[mp.mpf(1)], [mp.mpf(0), mp.mpf(1)]]
    for k in range(2, n):
        nxt = [mp.mpf(0)] * (k + 1)
        for i, c in enumerate(T[k - 1]):
            nxt[i + 1] += 2 * c
        for i, c in enumerate(T[k - 2]):
            nxt[i] -= c
        T.append(nxt)
    mono = [mp.mpf(0)] * n
    for k in range(n):
        for i, c in enumerate(T[k]):
            mono[i] += a[k] * c
    return mono


def fit_table(width, nseg, deg, pool):
    n = deg + 1
    nodes = [mp.cos(mp.pi * (j + mp.mpf(1) / 2) / n) for j in range(n)]
    pts = []
    for sgi in range(nseg):
        c = width * sgi + width / 2
        pts += [c + (width / 2) * s for s in nodes]
    vals = pool.map(_H, pts)
    segs = []
    for sgi in range(nseg):
        v = vals[sgi * n:(sgi + 1) * n]
        segs.append((_cheb_to_monomial([a[0] for a in v], deg), _cheb_to_monomial([a[1] for a in v], deg)))
    return segs


def _round(v, ctype):
    if ctype == "float":
        import numpy as np
        return float(np.float32(float(v)))
    return float(v)


def _check(width, nseg, deg, segs, ctype, pool, per_seg=24):
    """Max relative error of the rounded table (evaluated in the table precision with
    numpy, Horner order as in the kernels) against fresh reference points."""
    import numpy as np
    dt = np.float32 if ctype == "float" else np.float64
    ts = []
    for sgi in range(nseg):
        for k in range(per_seg):
            ts.append(float(width * sgi + width * (k + mp.mpf(1) / 3) / per_seg))
    ref = pool.map(_H, ts)
    err = [[0.0, 0.0] for _ in range(nseg)]
    for t, r in zip(ts, ref):
        sgi = min(int(t / float(width)), nseg - 1)
        s = dt((t - float(width * sgi + width / 2)) / float(width / 2))
        for f in range(2):
            acc = dt(0)
            for c in reversed(segs[sgi][f]):
                acc = dt(acc * s + dt(_round(c, ctype)))
            e = abs(float(acc) / float(r[f]) - 1.0)
            err[sgi][f] = max(err[sgi][f], e)
    return err


def main(out_path=None):
    here = os.path.dirname(os.path.abspath(__file__))
    out_path = out_path or os.path.join(os.path.dirname(here), "csrc", "synchro_coeffs.inc")
    lines = [
        "// Generated by paper_2008_10468_amd/fitgen/synchro_fit.py -- do not edit.",
        "// F(x) = t e^{-x} H_F(t), G(x) = t e^{-x} H_G(t), t = x^(1/3); per segment j of",
        "// width W in t a degree-D polynomial in s = (t - (j + 1/2) W) / (W / 2).",
        "// Layout: [segment][function F,G][coefficient c_0..c_D].  The includer defines",
        "// QED_SYN_STORAGE (e.g. __constant__ const) before including this file.",
        "",
    ]
    with mpc.Pool(min(16, os.cpu_count() or 1)) as pool:
        for name, ctype, width, nseg, deg in TABLES:
            segs = fit_table(width, nseg, deg, pool)
            err = _check(width, nseg, deg, segs, ctype, pool)
            worst = max(max(e) for e in err)
            print(f"{name}: {nseg} segments x degree {deg}, max rel err of H (table precision) {worst:.3e}",
                  file=sys.stderr)
            up = name.upper()
            lines.append(f"#define QED_SYN_{up}_NSEG {nseg}")
            lines.append(f"#define QED_SYN_{up}_NCOEF {deg + 1}")
            lines.append(f"#define QED_SYN_{up}_WIDTH {float(width)!r}")
            lines.append(f"#define QED_SYN_{up}_TMAX {float(width * nseg)!r}")
            lines.append(f"// max relative error of H over the table, in {ctype}: {worst:.3e}")
            lines.append(f"QED_SYN_STORAGE {ctype} qed_syn_{name}_coef[{nseg}][2][{deg + 1}] = {{")
            for sgi, (cf, cg) in enumerate(segs):
                def fmt(v):
                    if ctype == "float":
                        return repr(_round(v, ctype)) + "f"
                    return repr(float(v))
                lines.append(f"  {{ // segment {sgi}: t in [{float(width * sgi)}, {float(width * (sgi + 1))}],"
                             f" err F {err[sgi][0]:.2e} G {err[sgi][1]:.2e}")
                lines.append("    {" + ", ".join(fmt(c) for c in cf) + "},")
                lines.append("    {" + ", ".join(fmt(c) for c in cg) + "}},")
            lines.append("};")
            lines.append("")
    with open(out_path, "w") as f:
        f.write("\n".join(lines))
    print("wrote", out_path, file=sys.stderr)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else None)
