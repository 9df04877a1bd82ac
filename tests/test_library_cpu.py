"""CPU-side checks of the C-ABI library: it loads, exports every declared entry point,
its host-side thermodynamics agrees with the oracle's independent implementation,
and parameter validation rejects bad problem statements before touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import thermo as T

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "lbm2p.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_\w+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import paper_2112_01975_amd as P
    lib = ctypes.CDLL(P.lbm.LIB_PATH)
    names = _declared_symbols()
    assert len(names) >= 19
    for name in names:
        assert hasattr(lib, name), f"{name} not exported"
    assert set(names) == set(P.lbm.EXPORTED)


@pytest.mark.parametrize("eos,a,om,tr", [(0, 9 / 49, 0.0, 0.9), (0, 9 / 49, 0.0, 0.55), (1, 2 / 49, 0.344, 0.6),
                                         (1, 2 / 49, 0.344, 0.5), (2, 0.01, 0.344, 0.7), (3, 0.01, 0.0, 0.7),
                                         (5, 0.0, 0.0, 0.9), (5, 0.0, 0.0, 0.6), (6, 0.0, 0.0, 0.9), (6, 0.0, 0.0, 0.6)])
def test_host_coexistence_matches_oracle(eos, a, om, tr):
    import paper_2112_01975_amd as P
    p = P.Params(P.LBM_D3Q27, 4, 4, 4, eos, a, 2 / 21, 1.0, om, tr)
    rv, rl, ps, Tt = P.lbm_coexistence(p)
    fl = T.Fluid(eos, a, 2 / 21, tr, 1.0, om)
    ov, ol, ops = T.coexistence(fl)
    assert abs(rv / ov - 1) < 1e-10 and abs(rl / ol - 1) < 1e-10 and abs(ps / ops - 1) < 1e-9
    assert abs(Tt / (fl.G if eos in (T.SC1, T.SC2) else fl.T) - 1) < 1e-15
    k = P.lbm_kappa_for_width(p, 5.0)
    assert abs(k / T.kappa_for_width(fl, 5.0) - 1) < 1e-8
    p.kappa = k
    assert abs(P.lbm_surface_tension(p) / T.surface_tension(fl, k) - 1) < 1e-7
    r = np.linspace(0.5 * ov, min(1.5 * ol, 0.99 * (fl.rho_max if hasattr(fl, "rho_max") else 1.5 * ol)), 7)
    assert np.allclose(P.lbm_eos_pressure(p, r), [fl.pressure(x) for x in r], rtol=1e-13, atol=0)


def test_no_loop_above_critical_temperature_is_a_domain_error():
    import paper_2112_01975_amd as P
    with pytest.raises(P.LbmError) as ei:
        P.lbm_coexistence(P.Params(P.LBM_D2Q9, 4, 4, 1, P.LBM_EOS_VDW, 9 / 49, 2 / 21, T_reduced=1.05))
    assert ei.value.code == P.LBM_E_DOMAIN


def _wall_rows(rows, q):
    """64x64 D2Q9 grid with solid rows at the given y, and every link fraction set to q."""
    m = np.zeros((64, 64), np.uint8)
    m[list(rows)] = 1
    return dict(mask=m.ravel(), rho_wall=1.0, link_q=np.full((9, 64 * 64), q))


@pytest.mark.parametrize("bad,msg", [
    (dict(lattice=7), "lattice"),
    (dict(nz=2), "nz == 1"),
    (dict(nx=0), "grid sizes"),
    (dict(tau_liquid=0.5), "tau_liquid"),
    (dict(kappa=-0.1), "kappa"),
    (dict(a=0.0), "EOS parameters"),
    (dict(T_reduced=0.0), "T_reduced"),
    (dict(precision=5), "precision"),
    (dict(eos=9), "equation of state"),
    (dict(tau_vapour=0.4), "tau_vapour"),
    (dict(tau_vapour=0.9, rho_liquid=1.0, rho_vapour=2.0), "variable viscosity"),
    (dict(mask=np.zeros(64 * 64, np.uint8), rho_wall=0.0), "rho_wall"),
    (dict(link_q=np.full((9, 64 * 64), 0.5)), "link_q needs a mask"),
    (_wall_rows((0,), 0.0), "(0, 1]"),
    (_wall_rows((0,), 1.5), "(0, 1]"),
    (_wall_rows((10, 12), 1.0), "1.01"),          # row 11 cut on both sides at q = 1
    (dict(lattice=1, nx=1400, ny=1400, nz=1400), "larger than 2^31"),
    # 1025 x 1427^2 fits below 2^31 nodes, but not with its rows padded to 1056
    (dict(lattice=1, nx=1025, ny=1427, nz=1427), "with its rows padded"),
    (dict(force_model=4), "force model"),
    (dict(force_model=2, force_g=(float("nan"), 0.0, 0.0, 0.0)), "force_g"),
])
def test_create_rejects_bad_parameters_without_gpu(bad, msg):
    import paper_2112_01975_amd as P
    kw = dict(lattice=P.LBM_D2Q9, nx=64, ny=64, nz=1)
    kw.update(bad)
    p = P.Params(**kw)
    with pytest.raises(P.LbmError) as ei:
        P.lbm_create(p)
    assert ei.value.code == P.LBM_E_INVAL
    assert msg in str(ei.value)
    assert msg in P.lbm_last_error(None)


def test_batch_rejects_interpolated_walls_without_gpu():
    import paper_2112_01975_amd as P
    p = P.Params(P.LBM_D2Q9, 64, 64, 1, **_wall_rows((0,), 0.5))
    with pytest.raises(P.LbmError) as ei:
        P.lbm_batch_create([p])
    assert ei.value.code == P.LBM_E_INVAL and "not supported by the batch" in str(ei.value)


@pytest.mark.parametrize("lattice,dims", [(0, (32768, 32768, 1)), (1, (1024, 1024, 600))])
def test_batch_rejects_cases_past_its_32_bit_field_offsets_without_gpu(lattice, dims):
    # the batch kernels address a case's fields at a N + n and step blocks by about N in
    # 32-bit ints: cases with (D + 1) N >= 2^31 are rejected before any device use
    import paper_2112_01975_amd as P
    nx, ny, nz = dims
    small = P.Params(P.LBM_D2Q9, 16, 4, 1)
    with pytest.raises(P.LbmError) as ei:
        P.lbm_batch_create([small, P.Params(lattice, nx, ny, nz)])
    assert ei.value.code == P.LBM_E_INVAL and "case 1: too large for the batch" in str(ei.value)


def test_velocity_sets_are_the_full_stencils():
    # D2Q9 / D3Q27 are the tensor products of {-1, 0, 1} per axis (Sec. 2.3: the D3Q27 set, and
    # D2Q9 as its reduction without the z component); the rest velocity comes first and every
    # velocity has its opposite
    import itertools
    import paper_2112_01975_amd as P
    for lattice, D, Q in ((P.LBM_D2Q9, 2, 9), (P.LBM_D3Q27, 3, 27)):
        c = np.asarray(P.lbm_velocities(lattice))
        assert c.shape == (Q, 3)
        assert (c[0] == 0).all()
        assert set(map(tuple, c[:, :D].tolist())) == set(itertools.product((-1, 0, 1), repeat=D))
        if D == 2:
            assert (c[:, 2] == 0).all()
        rows = set(map(tuple, c.tolist()))
        assert all(tuple(-v for v in r) in rows for r in rows)


def test_bench_refuses_more_than_one_gpu():
    # one GPU: --gpus N > 1 exits with a message before touching a device
    import json
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_profile_summaries_from_counter_files(tmp_path):
    # the profile summaries: traffic scaled by the copy probe's own counter reading, and busy
    # fractions over one XCD's active cycles (GRBM_GUI_ACTIVE is summed over the XCDs)
    from paper_2112_01975_amd import profsum
    hdr = '"Kernel_Name","Counter_Name","Counter_Value"\n'
    f = tmp_path / "fetch.csv"
    w = tmp_path / "write.csv"
    # copy of 1 MiB reads 512 KiB by the counter (factor 2), writes 1024 KiB (factor 1)
    f.write_text(hdr + '"k_copy<1>","FETCH_SIZE",512\n"k_fused3<float>","FETCH_SIZE",100\n'
                 '"k_fused3<float>","FETCH_SIZE",300\n')
    w.write_text(hdr + '"k_copy<1>","WRITE_SIZE",1024\n"k_fused3<float>","WRITE_SIZE",50\n')
    d = {}
    for line in profsum.traffic(str(f), str(w), "k_fused3", 1 << 20, "cmd").splitlines():
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            d[k.strip()] = v.strip()
    assert float(d["fetch_bytes_per_launch"]) == 200 * 1024 * 2
    assert float(d["write_bytes_per_launch"]) == 50 * 1024
    c = tmp_path / "pass" / "run_counter_collection.csv"
    c.parent.mkdir()
    c.write_text(hdr + '"k_fused3<float>","GRBM_GUI_ACTIVE",8000\n"k_fused3<float>","TA_BUSY_avr",750\n'
                 '"k_fused3<float>","TD_TD_BUSY_sum",176000\n"k_other","TA_BUSY_avr",1\n')
    out = profsum.counters("k_fused3", 256, 8, [str(c)], "cmd")
    assert "TA_BUSY_avr_frac_of_active_cycles: 0.7500" in out
    assert "TD_TD_BUSY_sum_frac_of_active_cycles: 0.6875" in out
