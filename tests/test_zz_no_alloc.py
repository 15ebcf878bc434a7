"""sg_solve_static (scratch in a static device array, no allocation) against
sg_solve through the C ABI: bit-identical results on two calls in a row, the
second on a smaller problem (the array keeps the first call's contents), and
a clear refusal of a problem whose scratch exceeds the array."""

import ctypes

import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu


def _run(spec, seed):
    import paper_2606_09688_amd as sg
    data = workloads.random_data(spec, seed)
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")
    sv = sg.SparseGridWave(*spec.args())
    f, u0, v0 = dev(data["f"]), dev(data["u0"]), dev(data["v0"])
    print("no-alloc case", spec, flush=True)
    U_ref = sv.solve(f, u0, v0)
    U_st = sv.solve(f, u0, v0, static=True)
    torch.cuda.synchronize()
    return sv, U_ref, U_st


def test_static_scratch_matches_sg_solve_twice():
    big = workloads.Spec(2, [1.0, 0.8], [2, 2], [1.0, 1.0, 1.0, 1.0], 1.0, 8)
    small = workloads.Spec(2, [1.0, 1.0], [1, 1], [1.3], 0.7, 5)
    for spec, seed in ((big, 1), (small, 2)):
        sv, U_ref, U_st = _run(spec, seed)
        assert torch.equal(U_st, U_ref), spec
        sv.close()


def test_static_scratch_one_dimensional_variable_speed():
    spec = workloads.Spec(1, [1.0], [4], [1.0, 0.6, 1.7, 0.9], 1.0, 9)
    sv, U_ref, U_st = _run(spec, 3)
    assert torch.equal(U_st, U_ref)
    sv.close()


def test_static_scratch_refuses_oversized_problem():
    import paper_2606_09688_amd as sg
    from paper_2606_09688_amd import binding
    spec = workloads.Spec(2, [1.0, 1.0], [1, 1], [1.0], 1.0, 11)
    print("no-alloc refusal", spec, flush=True)
    sv = sg.SparseGridWave(*spec.args())
    # the size check precedes every launch: the data pointers are not read
    t = torch.zeros(4, dtype=torch.float64, device="cuda:0")
    p = ctypes.c_void_p(t.data_ptr())
    st = binding.lib().sg_solve_static(sv._h, p, p, p, ctypes.c_void_p(t[2:].data_ptr()),
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    msg = binding.lib().sg_last_error().decode()
    assert st == -4, (st, msg)
    assert "bytes" in msg and "static" in msg, msg
    sv.close()
