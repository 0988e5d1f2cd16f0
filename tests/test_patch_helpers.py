"""Host check of the residual kernel's patch-interpolant helpers.

The local-projection pass of the general residual evaluates the patch
interpolant pi v (the Q1 function of the coarse cell that holds a fine cell)
directly at the fine cell's Gauss points, and tests against the patch's
corner functions directly, instead of interpolating to the cell's vertices
first.  Both routes compute the same quantities in exact arithmetic.  This
test compiles the helper section of the kernel source for the host (the
helpers are plain arithmetic) and checks, for every cell offset in its patch:

* values and physical gradients of pi v at the Gauss points agree with
  pi_vertices followed by eval_val / eval_vg to FP32 rounding;
* the corner integrals agree with integrate followed by pi_transpose;
* on exact Q1 data both routes reproduce the trilinear function's values and
  gradient (a closed form), so neither route can drift from the definition.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2307_14837_amd", "csrc", "residual.hip")

DRIVER = r"""
#include <cmath>
#include <cstdio>
#include <random>
#define __device__
#define __host__
#define __forceinline__ inline
using std::fmaf;
namespace dnnmg {
#include "helpers.inc"
}
using namespace dnnmg;
int main() {
    std::mt19937 rng(7);
    std::uniform_real_distribution<float> U(-1.f, 1.f);
    double ev = 0, eg = 0, ec = 0, eq = 0;
    const float ih0 = 3.f, ih1 = 5.f, ih2 = 7.f;
    for (int trial = 0; trial < 4000; ++trial) {
        const int ox = trial & 1, oy = (trial >> 1) & 1, oz = (trial >> 2) & 1;
        float c[8], G0[8], G1[8], G2[8];
        for (int j = 0; j < 8; ++j) { c[j] = U(rng); G0[j] = U(rng); G1[j] = U(rng); G2[j] = U(rng); }
        float sx[2], sy[2], sz[2];
        patch_coords(ox, sx); patch_coords(oy, sy); patch_coords(oz, sz);
        float pw[8], vr[8], t[8], g0[8], g1[8], g2[8];
        pi_vertices(c, ox, oy, oz, pw);
        eval_val(pw, vr);
        eval_vg(pw, ih0, ih1, ih2, t, g0, g1, g2);
        float v[8], GX[4], GY[4], GZ[4];
        patch_val(c, sx, sy, sz, v);
        patch_grad(c, sx, sy, sz, ih0, ih1, ih2, GX, GY, GZ);
        for (int q = 0; q < 8; ++q) {
            const int qa = q & 1, qb = (q >> 1) & 1, qc = q >> 2;
            ev = fmax(ev, fabs(v[q] - vr[q]));
            eg = fmax(eg, fabs(GX[qb + 2 * qc] - g0[q]) / ih0);
            eg = fmax(eg, fabs(GY[qa + 2 * qc] - g1[q]) / ih1);
            eg = fmax(eg, fabs(GZ[qa + 2 * qb] - g2[q]) / ih2);
            // closed form: trilinear interpolation of the corners at the
            // coarse coordinates of the Gauss point, in double
            const double X = sx[qa], Y = sy[qb], Z = sz[qc];
            double f = 0, fx = 0, fy = 0, fz = 0;
            for (int j = 0; j < 8; ++j) {
                const int A = j & 1, B = (j >> 1) & 1, C = j >> 2;
                const double lx = A ? X : 1 - X, ly = B ? Y : 1 - Y, lz = C ? Z : 1 - Z;
                const double dx = A ? 1 : -1, dy = B ? 1 : -1, dz = C ? 1 : -1;
                f += c[j] * lx * ly * lz;
                fx += c[j] * dx * ly * lz * 0.5 * ih0;
                fy += c[j] * lx * dy * lz * 0.5 * ih1;
                fz += c[j] * lx * ly * dz * 0.5 * ih2;
            }
            eq = fmax(eq, fabs(v[q] - f));
            eq = fmax(eq, fabs(GX[qb + 2 * qc] - fx) / ih0);
            eq = fmax(eq, fabs(GY[qa + 2 * qc] - fy) / ih1);
            eq = fmax(eq, fabs(GZ[qa + 2 * qb] - fz) / ih2);
        }
        float zero[8] = {0}, cv[8], cr[8], cd[8];
        integrate<true, true, true>(zero, G0, G1, G2, ih0, ih1, ih2, cv);
        pi_transpose(cv, ox, oy, oz, cr);
        patch_integrate_grad(G0, G1, G2, sx, sy, sz, ih0, ih1, ih2, cd);
        for (int j = 0; j < 8; ++j) ec = fmax(ec, fabs(cd[j] - cr[j]) / ih2);
    }
    printf("%.3e %.3e %.3e %.3e\n", ev, eg, ec, eq);
    return 0;
}
"""


def _helpers_section():
    src = open(SRC).read()
    start = src.index("constexpr float GLO")
    end = src.index("// ------------------------------------------------------------ kernel ------")
    return src[start:end]


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_patch_interpolant_routes_agree(tmp_path):
    (tmp_path / "helpers.inc").write_text(_helpers_section())
    (tmp_path / "t.cpp").write_text(DRIVER)
    exe = tmp_path / "t"
    subprocess.run(["g++", "-O1", "-ffp-contract=off", "-std=c++17", "-o", str(exe), str(tmp_path / "t.cpp")],
                   check=True, cwd=tmp_path)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    ev, eg, ec, eq = map(float, out)
    # inputs are O(1); every route is a handful of FP32 roundings
    assert ev < 1e-6, ev
    assert eg < 1e-6, eg
    assert ec < 2e-6, ec
    assert eq < 1e-6, eq
