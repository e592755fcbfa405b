"""Error paths and workspace ownership on the GPU.

- MP_ENOMEM through the allocation test hook (MP_FAIL_ALLOC=1): the call
  fails cleanly and the library works again once the hook is off.
- Calls on different streams own different workspaces: two streams with
  interleaved, unsynchronised calls give the same profiles as one stream.
"""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _note(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1901_05708_amd as m
    m.load()
    return m


def test_out_of_memory_hook_and_recovery(mp, monkeypatch):
    import torch
    rng = np.random.default_rng(3)
    T = torch.as_tensor(np.cumsum(rng.standard_normal(6000)), device="cuda")
    ref_P, ref_I = mp.acamp(T, 64, R=512)
    torch.cuda.synchronize()
    _note("allocation hook on a fresh stream")
    s = torch.cuda.Stream()     # a stream without a workspace yet
    monkeypatch.setenv("MP_FAIL_ALLOC", "1")
    with pytest.raises(mp.MpError) as ei:
        mp.acamp(T, 64, R=512, stream=s)
    assert ei.value.code == mp.MP_ENOMEM
    monkeypatch.delenv("MP_FAIL_ALLOC")
    P, I = mp.acamp(T, 64, R=512, stream=s)
    s.synchronize()
    assert torch.equal(P, ref_P) and torch.equal(I, ref_I)
    mp.load().mp_release()
    P, I = mp.acamp(T, 64, R=512)
    torch.cuda.synchronize()
    assert torch.equal(P, ref_P) and torch.equal(I, ref_I)


def test_two_streams_do_not_share_a_workspace(mp):
    """Interleaved calls on two streams, no synchronisation between them
    until the end: each stream's results equal the same calls made one at a
    time. Sizes differ so that the workspaces would move if shared."""
    import torch
    rng = np.random.default_rng(11)
    series = [np.cumsum(rng.standard_normal(n)) for n in (30000, 9000, 41000, 12000)]
    Ts = [torch.as_tensor(x, device="cuda") for x in series]
    m = 96
    ref = []
    for k, T in enumerate(Ts):
        fn = mp.acamp if k % 2 == 0 else mp.aamp
        P, I = fn(T, m, R=1024)
        torch.cuda.synchronize()
        ref.append((P.clone(), I.clone()))
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    _note("interleaved calls on two streams")
    out = []
    for rep in range(3):
        for k, T in enumerate(Ts):
            fn = mp.acamp if k % 2 == 0 else mp.aamp
            st = s1 if (k + rep) % 2 == 0 else s2
            with torch.cuda.stream(st):
                P, I = fn(T, m, R=1024, stream=st, validate=False)
            out.append((k, st, P, I))
    s1.synchronize()
    s2.synchronize()
    for k, st, P, I in out:
        assert torch.equal(I, ref[k][1]), f"series {k}: indices differ"
        assert torch.equal(P, ref[k][0]), f"series {k}: values differ"
