"""qed_emit_noalloc (the library's static per-device scratch instead of a caller workspace)
against qed_emit with a workspace, through the C ABI: same inputs, bit-identical leptons,
photons and counters, on two calls in a row (the second on a smaller set, so the scratch holds
the first call's contents when the second starts), in both precisions."""
import math

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    import paper_2511_08929_amd as q
    q.lib()
    return q


def _inputs(n, seed):
    rng = np.random.default_rng(seed)
    d = synth.random_unit_vectors(rng, n)
    g = np.exp(rng.uniform(math.log(300.0), math.log(8000.0), n))
    p = d * np.sqrt(g * g - 1)
    s = synth.random_unit_vectors(rng, n) * np.where(rng.random(n) < 0.2, rng.uniform(0, 1, n), 1.0)
    x = np.stack([rng.uniform(0, 200, n), rng.uniform(-5, 5, n), rng.uniform(-5, 5, n)])
    return x, p, s


def _run(q, tab, dtype, x, p, s, step, use_noalloc, cap):
    import torch
    n = p.shape[1]
    e = q.LeptonBuffers(0, cap, dtype, track=(True, True, True))
    g = q.PhotonBuffers(2 * cap, dtype, track=(True, True, True))
    e.load(x, p, s)
    ctr = q.new_counters()
    f = q.make_fields(q.QED_FIELD_PLANE_LP, E0=(0.0, 20.0, 0.0), B0=(0.0, 0.0, 60.0), a0=300.0, phase_len=400.0)
    sp = q.make_step(0.2, synth.EPS_R, step=step, t=step * 0.2, seed=11, flags=q.QED_ALL & ~q.QED_PAIR)
    for k in range(2):                         # two steps on the same set
        sp.step, sp.t = step + k, (step + k) * 0.2
        if use_noalloc:
            q.qed_emit_noalloc(tab, e, f, sp, g, ctr)
        else:
            ws = q.new_workspace(q.qed_workspace_size(cap))
            q.qed_emit(tab, e, f, sp, g, ctr, ws)
    torch.cuda.synchronize()
    assert e.n() == n
    return e.arrays(), g.arrays(), q.counters_dict(ctr)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_equals_workspace_call(q, prec):
    import torch
    tab = q.Tables(precision=q.QED_F64 if prec == "fp64" else q.QED_F32)
    dtype = torch.float64 if prec == "fp64" else torch.float32
    for n, cap, seed, step in ((40_000, 41_000, 3, 7), (1_500, 1_700, 4, 9)):      # the second call is smaller
        x, p, s = _inputs(n, seed)
        a = _run(q, tab, dtype, x, p, s, step, True, cap)
        b = _run(q, tab, dtype, x, p, s, step, False, cap)
        assert a[2] == b[2] and a[2]["n_emit"] > 50, (a[2], b[2])
        for u, v in zip(a[0], b[0]):
            assert np.array_equal(u, v)
        for u, v in zip(a[1], b[1]):
            assert np.array_equal(u, v)
        print(f"{prec} n={n}: {a[2]['n_emit']} photons, bit-identical")


def test_noalloc_rejects_capacity_beyond_the_scratch(q):
    """A set larger than the static scratch is rejected on the host before anything is enqueued."""
    import ctypes as C

    import torch
    tab = q.Tables(precision=q.QED_F32)
    e = q.LeptonBuffers(0, 8, torch.float32, track=(False, False, False))
    g = q.PhotonBuffers(8, torch.float32, track=(False, False, False))
    v = q.Leptons()
    C.pointer(v)[0] = e.view()
    v.capacity = q.QED_NOALLOC_MAX_LEPTONS + 1
    f, sp, ctr = q.make_fields(), q.make_step(0.1, synth.EPS_R), q.new_counters()
    st = q.lib().qed_emit_noalloc(tab.handle, C.byref(v), C.byref(f), C.byref(sp), C.byref(g.view()),
                                  C.c_void_p(ctr.data_ptr()), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == q.QED_ERR_CAPACITY
    assert b"static scratch maximum" in q.lib().qed_last_error()
    torch.cuda.synchronize()
    assert q.counters_dict(ctr) == {k: 0 for k in q.COUNTER_NAMES}
