"""One handle used from several host threads at once, each on its own HIP
stream (and so its own workspace): results match the oracle and no exchange
wait times out."""
import threading

import numpy as np
import pytest
import torch

import oracle
from paper_2609_01864_amd import credit as C
from paper_2609_01864_amd import inputs as I

pytestmark = pytest.mark.gpu


def test_concurrent_calls_from_threads(lib_built):
    h = C.Handle(0, load_default_model=False)
    M, N = 40, 25000
    errors = []

    def work(tid):
        try:
            s = torch.cuda.Stream()
            x32 = I.softmax_rows(M, N, seed=300 + tid).astype(np.float32)
            ref = oracle.softmax_fwd(x32.astype(np.float64))
            with torch.cuda.stream(s):
                x = torch.from_numpy(x32).cuda()
                for it in range(6):
                    plan = C.plan("split", 2 if (it + tid) % 2 else 4)
                    y, _ = C.softmax_fwd(x, p=plan, h=h)
                    s.synchronize()
                    err = np.max(np.abs(y.double().cpu().numpy() - ref))
                    if err > 2e-6:
                        errors.append((tid, it, err))
        except Exception as e:  # reported below
            errors.append((tid, repr(e)))

    threads = [threading.Thread(target=work, args=(t,)) for t in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    try:
        assert not any(t.is_alive() for t in threads)
        assert not errors, errors
        assert h.check_errors() == C.OK
    finally:
        h.close()


def test_concurrent_full_size_split_launches_on_two_streams(lib_built):
    # Two split-row launches whose grids each fill the GPU, issued at the same
    # time on two streams: the library orders them (one fence event per
    # device), so neither can hold part of the GPU while waiting for the
    # other's slots.  Every result equals the same call made alone (the split
    # kernel is deterministic) and no exchange wait gives up.
    h = C.Handle(0, load_default_model=False)
    M, N = 4096, 65536
    plan = C.plan("split", 8)
    assert h.geometry(C.SOFTMAX, C.FWD, C.F32, M, N, plan)["grid"] >= 256  # a full-GPU grid
    xs = [torch.from_numpy(I.softmax_rows(M, N, seed=400 + t).astype(np.float32)).cuda() for t in range(2)]
    alone = [C.softmax_fwd(x, p=plan, h=h)[0] for x in xs]
    torch.cuda.synchronize()
    errors = []
    barrier = threading.Barrier(2)

    def work(tid):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                barrier.wait()
                for it in range(8):
                    y, _ = C.softmax_fwd(xs[tid], p=plan, h=h)
                    s.synchronize()
                    if not torch.equal(y, alone[tid]):
                        errors.append((tid, it, "differs from the call made alone"))
        except Exception as e:  # reported below
            errors.append((tid, repr(e)))

    threads = [threading.Thread(target=work, args=(t,)) for t in range(2)]
    print("[threads] two full-size split launches", flush=True)
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    try:
        assert not any(t.is_alive() for t in threads)
        assert not errors, errors
        assert h.check_errors() == C.OK
    finally:
        h.close()
