"""lbm_moments_noalloc (device outputs, static per-device scratch) against lbm_moments.

Both entry points run the same moment and output kernels and the same reduction tree, so
the fields and totals agree bit for bit; the no-alloc call writes device buffers owned by
the caller and keeps its partial rows in the library's static scratch array, which keeps
the previous call's contents: two calls in a row, the second on a smaller grid, must each
match lbm_moments of their own state.
"""
import numpy as np
import pytest

from tests.gpu_cases import Case, drop_case_inputs

pytestmark = pytest.mark.gpu


def _device_moments(torch, P, s, D, N, fields=(True, True, True)):
    rho = torch.full((N,), float("nan"), dtype=torch.float64, device="cuda:0")
    U = torch.full((D, N), float("nan"), dtype=torch.float64, device="cuda:0")
    tot = torch.full((5,), float("nan"), dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    P.lbm_moments_noalloc(s.ctx, rho.data_ptr() if fields[0] else None, U.data_ptr() if fields[1] else None,
                          tot.data_ptr() if fields[2] else None)
    P.lbm_set_stream(s.ctx, None)   # waits for the context stream
    return rho.cpu().numpy(), U.cpu().numpy(), tot.cpu().numpy()


def _state(P, case, precision, steps, seed):
    rho0, u0 = drop_case_inputs(case, min(case.nx, case.ny) / 4, 4.0, 1e-4, seed)
    s = P.Simulation(case.params(precision))
    s.init(rho0, u0)
    s.step(steps)
    return s


def _same(P, torch, s, case):
    D, N = case.lattice, case.N
    r_h, U_h, t_h = s.moments()
    r_d, U_d, t_d = _device_moments(torch, P, s, D, N)
    print(f"case {case.lattice}D {case.nx}x{case.ny}x{case.nz}: totals {t_d}", flush=True)
    assert np.array_equal(r_d, r_h), "rho differs from lbm_moments"
    assert np.array_equal(U_d.reshape(D, N), U_h.reshape(D, N)), "U differs from lbm_moments"
    assert np.array_equal(t_d[:4], t_h), f"totals {t_d[:4]} vs {t_h}"
    assert t_d[4] == 0.0


def test_noalloc_matches_moments_two_calls_second_smaller():
    import torch

    import paper_2112_01975_amd as P
    # padded rows (nx 70 -> pitch 96), FP64 D3Q27 with the single-pass step, then a smaller
    # unpadded FP32 D2Q9 grid: the second call's tree is shorter than the first's
    big = Case(3, 70, 40, 36)
    small = Case(2, 33, 17)
    with _state(P, big, 0, 6, 1101) as s:
        _same(P, torch, s, big)
    with _state(P, small, 1, 9, 1102) as s:
        _same(P, torch, s, small)


def test_noalloc_nullable_outputs():
    import torch

    import paper_2112_01975_amd as P
    for case in (Case(2, 100, 30), Case(2, 40, 30)):   # padded and unpadded rows
        with _state(P, case, 0, 5, 1103) as s:
            r_h, U_h, t_h = s.moments()
            D, N = case.lattice, case.N
            for fields in ((True, False, False), (False, True, False), (False, False, True), (False, False, False)):
                r_d, U_d, t_d = _device_moments(torch, P, s, D, N, fields)
                if fields[0]:
                    assert np.array_equal(r_d, r_h)
                else:
                    assert np.isnan(r_d).all()      # untouched
                if fields[1]:
                    assert np.array_equal(U_d.reshape(D, N), U_h.reshape(D, N))
                else:
                    assert np.isnan(U_d).all()
                if fields[2]:
                    assert np.array_equal(t_d[:4], t_h)
                else:
                    assert np.isnan(t_d).all()


def test_noalloc_scratch_limit():
    import torch

    import paper_2112_01975_amd as P
    # the D2Q9 moment pass has ceil(nx/64) ceil(ny/4) workgroups; 209,610 of them fit the
    # 8 MiB scratch with the reduction tree's rows, 209,611 do not
    ok = Case(2, 8, 4 * 209610)
    with P.Simulation(ok.params(1)) as s:
        rng = np.random.default_rng(1104)
        rho0 = 0.3 + 0.01 * rng.random(ok.N)
        s.init(rho0, None)
        _same(P, torch, s, ok)
    over = Case(2, 8, 4 * 209611)
    with P.Simulation(over.params(1)) as s:
        with pytest.raises(P.LbmError) as e:
            P.lbm_moments_noalloc(s.ctx, None, None, None)
        assert e.value.code == P.LBM_E_INVAL and "scratch" in str(e.value)


def test_noalloc_captured_in_a_graph_replays_match_eager():
    # the entry point only enqueues kernels on the context stream (no allocation, memset or wait),
    # so it can be captured: a graph of one call, replayed after eager steps on the same stream,
    # gives lbm_moments of the state at each replay, bit for bit (padded rows: the output pass,
    # the staging and the repack are all in the graph). The graph holds the lattice that was
    # current at capture and the context alternates its two lattices every step, so the replays
    # come after even numbers of steps
    import torch

    import paper_2112_01975_amd as P
    case = Case(2, 70, 30)
    with _state(P, case, 0, 5, 1105) as s:
        D, N = case.lattice, case.N
        rho = torch.zeros(N, dtype=torch.float64, device="cuda:0")
        U = torch.zeros((D, N), dtype=torch.float64, device="cuda:0")
        tot = torch.zeros(5, dtype=torch.float64, device="cuda:0")
        stream = torch.cuda.Stream()
        P.lbm_set_stream(s.ctx, stream.cuda_stream)
        try:
            torch.cuda.synchronize()
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph, stream=stream):
                P.lbm_moments_noalloc(s.ctx, rho.data_ptr(), U.data_ptr(), tot.data_ptr())
            for rep in range(3):
                P.lbm_step(s.ctx, 8)                      # eager work between the replays
                with torch.cuda.stream(stream):
                    graph.replay()
                stream.synchronize()
                r_h, U_h, t_h = s.moments()
                print(f"replay {rep}: totals {tot.cpu().numpy()}", flush=True)
                assert np.array_equal(rho.cpu().numpy(), r_h), rep
                assert np.array_equal(U.cpu().numpy().reshape(D, N), U_h.reshape(D, N)), rep
                assert np.array_equal(tot.cpu().numpy()[:4], t_h), rep
        finally:
            P.lbm_set_stream(s.ctx, None)
