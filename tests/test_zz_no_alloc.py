"""qubo_bf_solve_noalloc -- qubo_bf_solve with its workspace in the library's
static device array -- against qubo_bf_solve with a caller workspace, through
the C ABI: identical energies, masks and status on consecutive calls, each
sequence ending with a smaller instance than the one before (the array keeps
the previous call's contents).  The smaller instances are also checked
against the oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_2310_19373_amd import _lib, inputs

pytestmark = pytest.mark.gpu

_DT = {np.dtype(np.float32): _lib.QUBO_F32, np.dtype(np.int32): _lib.QUBO_I32,
       np.dtype(np.float64): _lib.QUBO_F64, np.dtype(np.int64): _lib.QUBO_I64}


def _call(L, Q, k, noalloc):
    n = Q.shape[0]
    dt = _DT[Q.dtype]
    print(f"{'noalloc' if noalloc else 'solve'} n={n} dtype={Q.dtype} k={k}", flush=True)
    Qd = torch.from_numpy(np.ascontiguousarray(Q)).cuda()
    edt = torch.float64 if dt in (_lib.QUBO_F32, _lib.QUBO_F64) else torch.int64
    en = torch.zeros(k, dtype=edt, device="cuda")
    masks = torch.zeros(k, dtype=torch.int64, device="cuda")
    status = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    if noalloc:
        rc = L.qubo_bf_solve_noalloc(Qd.data_ptr(), n, n, dt, k, en.data_ptr(), masks.data_ptr(), status.data_ptr(),
                                     stream)
    else:
        nbytes = L.qubo_bf_workspace_size(n, k, dt)
        assert 0 < nbytes <= _lib.NOALLOC_SCRATCH_BYTES
        ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        rc = L.qubo_bf_solve(Qd.data_ptr(), n, n, dt, k, en.data_ptr(), masks.data_ptr(), status.data_ptr(),
                             ws.data_ptr(), nbytes, stream)
    assert rc == 0, _lib.last_error()
    torch.cuda.synchronize()
    return en.cpu().numpy(), masks.cpu().numpy().astype(np.uint64), int(status.cpu()[0])


SEQUENCES = {
    "f32": [(lambda: inputs.random_f32(34, 901), 16), (lambda: inputs.random_f32(21, 902), 4)],
    "i32": [(lambda: inputs.random_i32(32, 903), 16), (lambda: inputs.random_i32(19, 904, lo=-2, hi=2), 5)],
    "mixed": [(lambda: inputs.random_f32(28, 905).astype(np.float64), 8),
              (lambda: inputs.random_i32(22, 906).astype(np.int64), 3),
              (lambda: inputs.random_f32(9, 907), 2)],
}


@pytest.mark.parametrize("name", sorted(SEQUENCES))
def test_noalloc_matches_solve_on_consecutive_calls(gpu_lib, name):
    L = gpu_lib
    seq = SEQUENCES[name]
    for i, (make, k) in enumerate(seq):
        Q = make()
        e0, m0, s0 = _call(L, Q, k, noalloc=False)
        e1, m1, s1 = _call(L, Q, k, noalloc=True)
        assert s0 == 0 and s1 == 0, (s0, s1)
        assert np.array_equal(m1, m0), (m1, m0)
        assert np.array_equal(e1, e0), (e1, e0)
        if i > 0:  # the smaller instances: against the oracle as well
            E, M = oracle.topk(Q, k)
            assert np.array_equal(m1, M) and np.array_equal(e1, E), (m1, M, e1, E)
