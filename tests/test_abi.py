"""The C ABI without a GPU: libjt.so loads, exports every function that
include/jt.h declares, the ctypes structs have the C layout, and the host-only
entry points behave (b_n against scipy; no device -> a clean error)."""
import ctypes
import os
import re
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "jt.h")


def _lib():
    from paper_2606_01547_amd import _native
    if not os.path.exists(_native.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return _native.load_library(), _native


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(jt_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_pipeline_calls():
    names = _declared()
    for n in ("jt_ray_shoot", "jt_source_sb", "jt_convolve", "jt_simulate_image", "jt_deflection",
              "jt_upload_subhalos", "jt_upload_psf"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib, _ = _lib()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", os.path.join(ROOT, "paper_2606_01547_amd", "libjt.so")],
                         capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r" T (jt_\w+)", out))
    assert set(_declared()) <= exported


def test_binding_declares_every_symbol():
    _, nat = _lib()
    assert set(_declared()) == set(nat._SIGS)


LAYOUT_C = r"""
#include <stdio.h>
#include <stddef.h>
#include "jt.h"
#define P(T) printf(#T " %zu\n", sizeof(T))
#define O(T, f) printf(#T "." #f " %zu\n", offsetof(T, f))
int main(void) {
  P(jt_grid); O(jt_grid, pixel_scale); O(jt_grid, y0);
  P(jt_sie); P(jt_shear);
  P(jt_nfw); O(jt_nfw, x); O(jt_nfw, alpha_Rs); O(jt_nfw, r_trunc);
  P(jt_point_masses); O(jt_point_masses, theta_E);
  P(jt_epl); O(jt_epl, gamma); O(jt_epl, cy);
  P(jt_lens); O(jt_lens, sie); O(jt_lens, shear); O(jt_lens, nfw); O(jt_lens, subhalo_handle); O(jt_lens, pm);
  O(jt_lens, has_epl); O(jt_lens, epl);
  P(jt_request); O(jt_request, sie); O(jt_request, subhalo_handle); O(jt_request, src); O(jt_request, lens_light);
  O(jt_request, psf_handle); O(jt_request, out); O(jt_request, has_epl); O(jt_request, epl);
  P(jt_sersic); P(jt_light); O(jt_light, c); O(jt_light, bn_exact); O(jt_light, n_gauss); O(jt_light, gauss);
  O(jt_light, n_core); O(jt_light, core); O(jt_light, shapelets);
  P(jt_gaussian); P(jt_core_sersic); O(jt_core_sersic, alpha); P(jt_shapelets); O(jt_shapelets, beta);
  O(jt_shapelets, coeff);
  P(jt_draws); O(jt_draws, sie); O(jt_draws, n_sub); O(jt_draws, sub_alpha_Rs); O(jt_draws, n_ll); O(jt_draws, ll);
  O(jt_draws, epl); O(jt_draws, sub_r_trunc);
  P(jt_server_stats); O(jt_server_stats, device_seconds); O(jt_server_stats, max_wait_seconds);
  P(jt_fit_problem); O(jt_fit_problem, lower); O(jt_fit_problem, n_sub); O(jt_fit_problem, sub_alpha_Rs);
  O(jt_fit_problem, psf); O(jt_fit_problem, k); O(jt_fit_problem, inv_var);
  P(jt_pso_cfg); O(jt_pso_cfg, inertia); O(jt_pso_cfg, seed); P(jt_lbfgs_cfg); O(jt_lbfgs_cfg, ftol);
  return 0;
}
"""


def test_ctypes_structs_match_c_layout(tmp_path):
    _, nat = _lib()
    src = tmp_path / "layout.c"
    src.write_text(LAYOUT_C)
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                    "-I", "/opt/rocm/include", str(src), "-o", str(exe)], check=True)
    got = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                              check=True).stdout.splitlines())
    m = {"jt_grid": nat.JtGrid, "jt_sie": nat.JtSie, "jt_shear": nat.JtShear, "jt_nfw": nat.JtNfw,
         "jt_point_masses": nat.JtPointMasses, "jt_lens": nat.JtLens, "jt_sersic": nat.JtSersic,
         "jt_light": nat.JtLight, "jt_draws": nat.JtDraws, "jt_server_stats": nat.JtServerStats,
         "jt_epl": nat.JtEpl, "jt_request": nat.JtRequest, "jt_fit_problem": nat.JtFitProblem,
         "jt_pso_cfg": nat.JtPsoCfg, "jt_lbfgs_cfg": nat.JtLbfgsCfg, "jt_gaussian": nat.JtGaussian,
         "jt_core_sersic": nat.JtCoreSersic, "jt_shapelets": nat.JtShapelets}
    for key, val in got.items():
        if "." in key:
            t, f = key.split(".")
            assert getattr(m[t], f).offset == int(val), key
        else:
            assert ctypes.sizeof(m[key]) == int(val), key


@pytest.mark.parametrize("n", [0.2, 0.5, 1.0, 2.0, 3.7, 4.0, 6.0, 10.0])
def test_exact_bn_matches_scipy(n):
    from scipy.special import gammaincinv
    _, nat = _lib()
    assert nat.sersic_bn(n, exact=True) == pytest.approx(float(gammaincinv(2 * n, 0.5)), rel=1e-13)
    assert nat.sersic_bn(n, exact=False) == pytest.approx(1.9992 * n - 0.3271, rel=1e-15)


def test_bn_rejects_out_of_range():
    _, nat = _lib()
    assert np.isnan(nat.sersic_bn(0.1, True)) and np.isnan(nat.sersic_bn(11.0, False))


def test_create_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    _, nat = _lib()
    with pytest.raises(nat.JtError) as ei:
        nat.Context(0)
    assert ei.value.status in (nat.JT_EDEVICE, nat.JT_EINVAL)


def test_convolve_auto_method_host_rule():
    _, nat = _lib()
    assert nat.convolve_auto_method(200, 200, 3) == 1        # tiny kernel: direct
    assert nat.convolve_auto_method(64, 64, 301) == 2        # beyond the direct limit: FFT
    assert nat.convolve_auto_method(3000, 10, 301) == 0      # neither path takes it
    assert nat.convolve_auto_method(2000, 2000, 101) == 1    # FFT size over 2048: direct
    assert nat.convolve_auto_method(10, 10, 4) == 0          # even kernel
    assert nat.convolve_auto_method(0, 10, 3) == 0


def test_counter_uniforms_match_the_oracle_generator():
    import oracle as O
    _, nat = _lib()
    for seed in (0, 1, 1234567, 2 ** 63 + 5):
        for i in (0, 1, 2, 1000, 2 ** 40 + 3):
            assert nat.uniform(seed, i) == O.uniform(seed, i)


def test_swarm_update_matches_the_oracle_step():
    import oracle as O
    _, nat = _lib()
    rng = np.random.default_rng(2)
    N, P = 7, 5
    lo, hi = -np.ones(P), 2.0 * np.ones(P)
    x = rng.uniform(-1, 2, (N, P))
    v = rng.normal(0, 0.8, (N, P))
    pbest = rng.uniform(-1, 2, (N, P))
    gbest = rng.uniform(-1, 2, P)
    for t in (1, 2, 9):
        ex, ev = O.pso_move(t, x, v, pbest, gbest, lo, hi, 11, 0.7298, 1.49618, 1.49618)
        gx, gv = x.copy(), v.copy()
        nat.pso_move(t, 11, 0.7298, 1.49618, 1.49618, lo, hi, gx, gv, pbest, gbest)
        np.testing.assert_allclose(gx, ex, rtol=1e-15, atol=1e-15)
        np.testing.assert_allclose(gv, ev, rtol=1e-15, atol=1e-15)
        assert np.all(gx >= lo) and np.all(gx <= hi)
        x, v = gx, gv
