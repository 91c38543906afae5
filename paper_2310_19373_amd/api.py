"""Python surface over the C ABI: device memory and streams come from PyTorch,
every computation runs in the HIP library.

* ``solve(Q, k)``                   k lowest states of one QUBO
* ``solve_range`` / ``merge_topk``  one prefix range of a solve / merge of such results
* ``solve_resumable``               a solve in checkpointed prefix-range pieces
* ``solve_batched(Qpad, ns, k)``    k lowest states of many QUBOs, one launch sequence
* ``BatchedSolver``                 the same with persistent buffers and optional
                                    HIP-graph capture/replay
* ``logz(Q, beta)``                 exact log-partition function, differentiable
* ``masks_to_bits(masks, n)``       uint64 masks (bit i = x_i) -> 0/1 matrix
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib
from ._lib import QuboError

__all__ = ["solve", "solve_batched", "BatchedSolver", "logz", "LogZ", "masks_to_bits", "QuboError",
           "UncertainError"]


class UncertainError(QuboError):
    """The float certificate could not prove the selection (ties closer than
    the float32 rounding bound)."""


_STATUS = {
    _lib.QUBO_ERR_INVALID_ARG: "invalid instance size",
    _lib.QUBO_ERR_NONFINITE: "Q or beta holds inf or NaN",
    _lib.QUBO_ERR_UNCERTAIN: "float certificate failed",
    _lib.QUBO_ERR_RANGE: "int64 Q with sum |Q_ij| beyond the exact range (2^50)",
    _lib.QUBO_ERR_OVERFLOW: "internal candidate slot overflow",
}


def _as_device(x, dtype=None, device=None):
    if isinstance(x, np.ndarray):
        x = torch.from_numpy(np.ascontiguousarray(x))
    if not isinstance(x, torch.Tensor):
        x = torch.as_tensor(x)
    dev = device if device is not None else (x.device if x.is_cuda else torch.device("cuda", torch.cuda.current_device()))
    if dtype is not None and x.dtype != dtype:
        x = x.to(dtype)
    return x.to(dev).contiguous()


_DTYPES = {torch.float32: _lib.QUBO_F32, torch.int32: _lib.QUBO_I32, torch.float64: _lib.QUBO_F64,
           torch.int64: _lib.QUBO_I64}


def _qdtype(t) -> int:
    dt = _DTYPES.get(t.dtype if isinstance(t, torch.Tensor) else t)
    if dt is None:
        raise TypeError("Q must be float32, int32, float64 or int64")
    return dt


def _energy_dtype(dt: int):
    return torch.float64 if dt in (_lib.QUBO_F32, _lib.QUBO_F64) else torch.int64


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _raise_status(status: torch.Tensor):
    st = status.cpu().numpy()
    bad = np.nonzero(st != 0)[0]
    if bad.size:
        code = int(st[bad[0]])
        msg = f"{_STATUS.get(code, 'error')} (instance {int(bad[0])}, {bad.size} affected)"
        if code == _lib.QUBO_ERR_UNCERTAIN:
            raise UncertainError(code, msg)
        raise QuboError(code, msg)


def _check_upper(Q: torch.Tensor):
    if torch.any(torch.tril(Q, -1) != 0).item():
        raise ValueError("Q must be upper triangular (entries below the diagonal are nonzero)")


def solve(Q, k: int = 1, *, check_lower: bool = True, retry_uncertain: bool = True, kprime: int = 0):
    """The k lowest states of f_Q(x) = x^T Q x over x in {0,1}^n.

    Q: (n, n) float32, int32, float64 or int64 tensor/array, upper triangular.
    Returns (energies, masks) on Q's GPU: float64 (float Q) or int64 (int Q),
    and int64 tensors holding the uint64 masks (bit i = x_i), ascending by
    (energy, mask).  Slots beyond 2^n hold +inf / INT64_MAX and mask -1.
    kprime: candidate list length (0: the library's default); a float solve
    whose certificate fails is repeated once with 64 when retry_uncertain.
    """
    Qd = _as_device(Q)
    if Qd.ndim != 2 or Qd.shape[0] != Qd.shape[1]:
        raise ValueError("Q must be square")
    if check_lower:
        _check_upper(Qd)
    n = Qd.shape[0]
    dt = _qdtype(Qd)
    L = _lib.lib()
    ws_bytes = L.qubo_bf_workspace_size_kp(n, k, kprime, dt)
    if ws_bytes == 0:
        raise ValueError(f"invalid arguments n={n}, k={k}, kprime={kprime}: {_lib.last_error()}")
    dev = Qd.device
    with torch.cuda.device(dev):
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
        en = torch.empty(k, dtype=_energy_dtype(dt), device=dev)
        masks = torch.empty(k, dtype=torch.int64, device=dev)
        status = torch.empty(1, dtype=torch.int32, device=dev)
        _lib.check(L.qubo_bf_solve_kp(Qd.data_ptr(), n, n, dt, k, kprime, en.data_ptr(), masks.data_ptr(),
                                      status.data_ptr(), ws.data_ptr(), ws_bytes, _stream(dev)))
        try:
            _raise_status(status)
        except UncertainError:
            if not retry_uncertain or dt not in (_lib.QUBO_F32, _lib.QUBO_F64) or kprime == 64:
                raise
            return solve(Qd, k, check_lower=False, retry_uncertain=False, kprime=64)
    return en, masks


def solve_range(Q, k: int, p_bits: int, p_begin: int, p_end: int, *, check_lower: bool = True):
    """The k lowest states among the masks whose top p_bits bits lie in
    [p_begin, p_end) -- one resumable piece of solve(Q, k).  Results of
    disjoint ranges combine with merge_topk into the result of solve.
    Returns (energies, masks) like solve; raises UncertainError if the float
    certificate fails for the range."""
    Qd = _as_device(Q)
    if Qd.ndim != 2 or Qd.shape[0] != Qd.shape[1]:
        raise ValueError("Q must be square")
    if check_lower:
        _check_upper(Qd)
    n = Qd.shape[0]
    dt = _qdtype(Qd)
    L = _lib.lib()
    ws_bytes = L.qubo_bf_range_workspace_size(n, k, dt, p_bits)
    if ws_bytes == 0:
        raise ValueError(f"invalid arguments n={n}, k={k}, p_bits={p_bits}: {_lib.last_error()}")
    dev = Qd.device
    with torch.cuda.device(dev):
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
        en = torch.empty(k, dtype=_energy_dtype(dt), device=dev)
        masks = torch.empty(k, dtype=torch.int64, device=dev)
        status = torch.empty(1, dtype=torch.int32, device=dev)
        _lib.check(L.qubo_bf_solve_range(Qd.data_ptr(), n, n, dt, k, p_bits, p_begin, p_end, en.data_ptr(),
                                         masks.data_ptr(), status.data_ptr(), ws.data_ptr(), ws_bytes, _stream(dev)))
        _raise_status(status)
    return en, masks


def merge_topk(results, k: int):
    """The k lowest (energy, mask) pairs over a list of (energies, masks)
    results of solve_range on disjoint ranges of one instance (device merge)."""
    if not results:
        raise ValueError("nothing to merge")
    en = torch.stack([r[0] for r in results]).contiguous()
    mk = torch.stack([r[1] for r in results]).contiguous()
    dev = en.device
    dt = _lib.QUBO_F32 if en.dtype == torch.float64 else _lib.QUBO_I32
    out_e = torch.empty(k, dtype=en.dtype, device=dev)
    out_m = torch.empty(k, dtype=torch.int64, device=dev)
    with torch.cuda.device(dev):
        _lib.check(_lib.lib().qubo_bf_merge_topk(en.shape[0], en.shape[1], en.data_ptr(), mk.data_ptr(), dt, k,
                                                 out_e.data_ptr(), out_m.data_ptr(), _stream(dev)))
    return out_e, out_m


def solve_resumable(Q, k: int, p_bits: int, checkpoint: str, *, max_ranges: int | None = None):
    """solve(Q, k) in 2^p_bits prefix-range pieces (solve_range), for long
    enumerations: after each piece the merged result of the finished pieces
    and the next prefix are written atomically to ``checkpoint`` (an .npz
    file), and a later call with the same Q, k and p_bits resumes from it.

    max_ranges bounds the pieces done by this call (None: all that remain).
    Returns (energies, masks, done, total) with the k lowest so far and the
    number of finished pieces; done == total means the result is final.
    """
    import hashlib
    import os

    Qd = _as_device(Q)
    if Qd.ndim != 2 or Qd.shape[0] != Qd.shape[1]:
        raise ValueError("Q must be square")
    _check_upper(Qd)
    n = Qd.shape[0]
    total = 1 << p_bits
    key = hashlib.sha256(Qd.cpu().numpy().tobytes()).hexdigest()
    meta = np.array([n, k, p_bits, _qdtype(Qd)], dtype=np.int64)
    dev = Qd.device
    done, best = 0, None
    if os.path.exists(checkpoint):
        with np.load(checkpoint, allow_pickle=False) as z:
            if str(z["q_sha256"]) != key or not np.array_equal(z["meta"], meta):
                raise ValueError(f"{checkpoint} belongs to another instance, k or p_bits")
            done = int(z["done"])
            if done:
                best = (torch.from_numpy(z["energies"]).to(dev), torch.from_numpy(z["masks"]).to(dev))
    stop = total if max_ranges is None else min(total, done + max_ranges)
    while done < stop:
        part = solve_range(Qd, k, p_bits, done, done + 1, check_lower=False)
        best = part if best is None else merge_topk([best, part], k)
        done += 1
        tmp = checkpoint + ".tmp.npz"
        np.savez(tmp, q_sha256=np.array(key), meta=meta, done=np.array(done), energies=best[0].cpu().numpy(),
                 masks=best[1].cpu().numpy())
        os.replace(tmp, checkpoint)
    if best is None:
        raise ValueError("no piece finished yet (max_ranges=0)")
    return best[0], best[1], done, total


class BatchedSolver:
    """Persistent buffers for repeated batched solves of one shape.

    ``run()`` enqueues the library's launch sequence; with ``graph=True`` the
    sequence is captured once into a HIP graph (no allocation, no host sync,
    no memset nodes inside) and later calls replay it.

    ``autotune=True``: the first ``run()`` picks the launch shape (outer bits
    per work unit, waves per CU, queue chunk) for the loaded batch with
    ``autotune.tune_batched`` -- or takes it from ``tune_cache`` (a JSON file
    keyed by the batch's size histogram) when it holds this workload -- and
    the solver then enqueues under that shape: with ``graph=True`` it is
    captured into the graph, else it is set around each enqueue.  The
    library's tuning knobs are process-wide; they are restored after each
    use, so other calls keep their own settings (calls from other threads
    while a solver enqueues would see the solver's shape).
    """

    def __init__(self, batch: int, nmax: int, k: int = 1, dtype=torch.float32, device=None, graph: bool = False,
                 autotune: bool = False, tune_cache: str | None = None):
        self.batch, self.nmax, self.k = batch, nmax, k
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.dt = _qdtype(dtype)
        L = _lib.lib()
        self.ws_bytes = L.qubo_bf_batched_workspace_size(batch, nmax, k, self.dt)
        if self.ws_bytes == 0:
            raise ValueError(f"invalid arguments: {_lib.last_error()}")
        d = self.device
        self.Q = torch.zeros((batch, nmax, nmax), dtype=dtype, device=d)
        self.ns = torch.zeros(batch, dtype=torch.int32, device=d)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=d)
        self.energies = torch.empty((batch, k), dtype=_energy_dtype(self.dt), device=d)
        self.masks = torch.empty((batch, k), dtype=torch.int64, device=d)
        self.status = torch.empty(batch, dtype=torch.int32, device=d)
        self.use_graph = graph
        self.graph = None
        self.autotune, self.tune_cache = autotune, tune_cache
        self.setting = None       # the tuned launch shape (knob name -> value), once tuned
        self.tune_result = None   # autotune.TuneResult when this solver ran the search

    def load(self, Qpad, ns):
        self.Q.copy_(_as_device(Qpad, self.Q.dtype, self.device))
        self.ns.copy_(_as_device(ns, torch.int32, self.device))

    def _tune(self):
        from . import autotune as at

        names = list(at.BATCHED_SPACE)
        sig = at.batched_signature(self.ns.cpu().numpy(), self.k, at._DT_NAMES[self.dt],
                                   torch.cuda.get_device_name(self.device))
        with at.keep_tuning(names):
            best = at.load_cached(self.tune_cache, sig) if self.tune_cache else None
            if best is None:
                self.tune_result = at.tune_batched(self.Q, self.ns, self.k, apply_best=False, cache=self.tune_cache)
                best = self.tune_result.best
        self.use_setting(best)

    def use_setting(self, setting: dict):
        """Enqueue under this launch shape from now on (knob name -> value,
        as autotune.BATCHED_SPACE); resizes the workspace if it needs to."""
        from . import autotune as at

        self.setting = dict(setting)
        with at.keep_tuning(list(self.setting)):
            at.apply(self.setting)
            nbytes = _lib.lib().qubo_bf_batched_workspace_size(self.batch, self.nmax, self.k, self.dt)
        if nbytes != self.ws_bytes:
            self.ws_bytes = nbytes
            self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.graph = None

    def _enqueue(self):
        L = _lib.lib()
        if self.setting is not None:
            from . import autotune as at

            with at.keep_tuning(list(self.setting)):
                at.apply(self.setting)
                return self._enqueue_now(L)
        return self._enqueue_now(L)

    def _enqueue_now(self, L):
        _lib.check(L.qubo_bf_solve_batched(self.batch, self.Q.data_ptr(), self.nmax, self.ns.data_ptr(), self.dt,
                                           self.k, self.energies.data_ptr(), self.masks.data_ptr(),
                                           self.status.data_ptr(), self.ws.data_ptr(), self.ws_bytes,
                                           _stream(self.device)))

    def run(self):
        with torch.cuda.device(self.device):
            if self.autotune and self.setting is None:
                self._tune()
            if not self.use_graph:
                self._enqueue()
                return
            if self.graph is None:
                s = torch.cuda.Stream(self.device)
                s.wait_stream(torch.cuda.current_stream(self.device))
                with torch.cuda.stream(s):
                    self._enqueue()  # warm-up outside capture (loads modules)
                torch.cuda.current_stream(self.device).wait_stream(s)
                torch.cuda.synchronize(self.device)
                self.graph = torch.cuda.CUDAGraph()
                with torch.cuda.graph(self.graph):
                    self._enqueue()
            self.graph.replay()

    def results(self, check: bool = True):
        if check:
            _raise_status(self.status)
        return self.energies, self.masks


def solve_batched(Qpad, ns, k: int = 1, *, check_lower: bool = True):
    """Independent k-lowest solves of many QUBOs, one launch sequence at the
    current launch shape (for repeated solves of one shape, a BatchedSolver
    with graph=True and autotune=True).

    Qpad: (batch, nmax, nmax) float32/int32/float64/int64, instance b in Qpad[b, :ns[b], :ns[b]].
    Returns (energies [batch, k], masks [batch, k]) on the GPU.
    """
    Qd = _as_device(Qpad)
    if Qd.ndim != 3 or Qd.shape[1] != Qd.shape[2]:
        raise ValueError("Qpad must be (batch, nmax, nmax)")
    if check_lower:
        _check_upper(Qd)
    nsd = _as_device(ns, torch.int32, Qd.device)
    batch, nmax = Qd.shape[0], Qd.shape[1]
    solver = BatchedSolver(batch, nmax, k, Qd.dtype, Qd.device)
    solver.Q = Qd
    solver.ns = nsd
    solver.run()
    return solver.results()


def masks_to_bits(masks, n: int) -> np.ndarray:
    """(..., ) uint64/int64 masks -> (..., n) uint8 matrix with x_i = bit i."""
    if isinstance(masks, torch.Tensor):
        masks = masks.detach().cpu().numpy()
    m = np.asarray(masks).astype(np.uint64)
    return ((m[..., None] >> np.arange(n, dtype=np.uint64)) & np.uint64(1)).astype(np.uint8)


def _logz_ws(batch, nmax, device):
    L = _lib.lib()
    nbytes = L.qubo_logz_workspace_size(batch, nmax)
    if nbytes == 0:
        raise ValueError(f"invalid arguments batch={batch}, nmax={nmax}: {_lib.last_error()}")
    return torch.empty(nbytes, dtype=torch.uint8, device=device), nbytes


class LogZ(torch.autograd.Function):
    """logZ_b = log sum_x exp(-beta_b x^T Q_b x) with its exact gradient.

    forward(Q [batch, nmax, nmax] float32, beta [batch] float32, ns [batch] int32)
    -> logZ [batch] float64.  backward re-enumerates every state (adjoint walk)
    and returns d/dQ (upper triangle incl. diagonal, zeros elsewhere) and d/dbeta.
    """

    @staticmethod
    def forward(ctx, Q, beta, ns):
        dev = Q.device
        batch, nmax = Q.shape[0], Q.shape[1]
        Qc = Q.detach().contiguous()
        bc = beta.detach().to(torch.float32).contiguous()
        nsc = ns.to(torch.int32).contiguous()
        out = torch.empty(batch, dtype=torch.float64, device=dev)
        status = torch.empty(batch, dtype=torch.int32, device=dev)
        ws, nbytes = _logz_ws(batch, nmax, dev)
        with torch.cuda.device(dev):
            _lib.check(_lib.lib().qubo_logz_fwd(batch, Qc.data_ptr(), nmax, nsc.data_ptr(), bc.data_ptr(),
                                                out.data_ptr(), status.data_ptr(), ws.data_ptr(), nbytes,
                                                _stream(dev)))
        _raise_status(status)
        ctx.save_for_backward(Qc, bc, nsc, out)
        return out

    @staticmethod
    def backward(ctx, g):
        Qc, bc, nsc, lz = ctx.saved_tensors
        dev = Qc.device
        batch, nmax = Qc.shape[0], Qc.shape[1]
        gq = torch.empty_like(Qc)
        gb = torch.empty(batch, dtype=torch.float32, device=dev)
        status = torch.empty(batch, dtype=torch.int32, device=dev)
        gl = g.detach().to(torch.float32).contiguous()
        ws, nbytes = _logz_ws(batch, nmax, dev)
        with torch.cuda.device(dev):
            _lib.check(_lib.lib().qubo_logz_bwd(batch, Qc.data_ptr(), nmax, nsc.data_ptr(), bc.data_ptr(),
                                                lz.data_ptr(), gl.data_ptr(), gq.data_ptr(), gb.data_ptr(),
                                                status.data_ptr(), ws.data_ptr(), nbytes, _stream(dev)))
        _raise_status(status)
        return gq, gb, None


def logz(Q, beta, ns=None, *, check_lower: bool = True):
    """Exact log-partition function log sum_x exp(-beta f_Q(x)), differentiable.

    Q: (n, n) or (batch, nmax, nmax) float32 tensor (CUDA or CPU, upper
    triangular: a nonzero lower triangle raises ValueError unless check_lower
    is False, in which case it is ignored); beta: float or (batch,) tensor;
    ns: instance sizes for a padded batch (default: all nmax).  Returns
    float64: a 0-d tensor for a single Q, else (batch,).
    """
    single = False
    if not isinstance(Q, torch.Tensor):
        Q = torch.as_tensor(np.asarray(Q))
    if Q.ndim == 2:
        Q = Q.unsqueeze(0)
        single = True
    if Q.dtype != torch.float32:
        raise TypeError("Q must be float32")
    if not Q.is_cuda:
        Q = Q.to("cuda")
    if check_lower:
        _check_upper(Q.detach())
    dev = Q.device
    batch, nmax = Q.shape[0], Q.shape[1]
    if not isinstance(beta, torch.Tensor):
        beta = torch.full((batch,), float(beta), dtype=torch.float32, device=dev)
    beta = beta.to(dev)
    if beta.ndim == 0:
        beta = beta.expand(batch)
    if ns is None:
        ns = torch.full((batch,), nmax, dtype=torch.int32, device=dev)
    ns = _as_device(ns, torch.int32, dev)
    out = LogZ.apply(Q, beta, ns)
    return out[0] if single else out


def logz_moments(Q, beta, ns=None):
    """logZ with the second moments of p(x) = exp(-beta f(x) - logZ).

    Returns (logz [batch] float64, moments [batch, nmax, nmax] float64 with
    E_p[x_i x_j] for i <= j < n (marginals E_p[x_i] on the diagonal, zeros
    elsewhere), mean_energy [batch] float64 = E_p[f]); a single (n, n) Q gives
    unbatched results.
    """
    single = False
    if not isinstance(Q, torch.Tensor):
        Q = torch.as_tensor(np.asarray(Q))
    if Q.ndim == 2:
        Q = Q.unsqueeze(0)
        single = True
    if Q.dtype != torch.float32:
        raise TypeError("Q must be float32")
    Q = _as_device(Q, torch.float32)
    _check_upper(Q)
    dev = Q.device
    batch, nmax = Q.shape[0], Q.shape[1]
    if not isinstance(beta, torch.Tensor):
        beta = torch.full((batch,), float(beta), dtype=torch.float32, device=dev)
    beta = beta.to(device=dev, dtype=torch.float32).reshape(-1).expand(batch).contiguous()
    nsd = torch.full((batch,), nmax, dtype=torch.int32, device=dev) if ns is None else _as_device(ns, torch.int32, dev)
    lz = LogZ.apply(Q, beta, nsd).detach()
    mom = torch.empty((batch, nmax, nmax), dtype=torch.float64, device=dev)
    mean = torch.empty(batch, dtype=torch.float64, device=dev)
    status = torch.empty(batch, dtype=torch.int32, device=dev)
    ws, nbytes = _logz_ws(batch, nmax, dev)
    with torch.cuda.device(dev):
        _lib.check(_lib.lib().qubo_logz_moments(batch, Q.data_ptr(), nmax, nsd.data_ptr(), beta.data_ptr(),
                                                lz.data_ptr(), mom.data_ptr(), mean.data_ptr(), status.data_ptr(),
                                                ws.data_ptr(), nbytes, _stream(dev)))
    _raise_status(status)
    if single:
        return lz[0], mom[0], mean[0]
    return lz, mom, mean


def marginals(Q, beta, ns=None):
    """E_p[x_i] under p(x) = exp(-beta f(x) - logZ): the diagonal of logz_moments."""
    _, mom, _ = logz_moments(Q, beta, ns)
    return torch.diagonal(mom, dim1=-2, dim2=-1)


def logz_sample(Q, beta, u, ns=None):
    """Exact samples of p(x) = exp(-beta f(x) - logZ) by inversion of the
    cumulative distribution in natural mask order.

    u: uniforms in [0, 1), shape [batch, nsamples] (or [nsamples] for a single
    (n, n) Q), float64; the caller owns the random stream.  Returns (masks
    [batch, nsamples] int64 -- bit i is x_i --, logz [batch] float64).
    """
    single = False
    if not isinstance(Q, torch.Tensor):
        Q = torch.as_tensor(np.asarray(Q))
    if Q.ndim == 2:
        Q = Q.unsqueeze(0)
        single = True
    if Q.dtype != torch.float32:
        raise TypeError("Q must be float32")
    Q = _as_device(Q, torch.float32)
    _check_upper(Q)
    dev = Q.device
    batch, nmax = Q.shape[0], Q.shape[1]
    if not isinstance(beta, torch.Tensor):
        beta = torch.full((batch,), float(beta), dtype=torch.float32, device=dev)
    beta = beta.to(device=dev, dtype=torch.float32).reshape(-1).expand(batch).contiguous()
    nsd = torch.full((batch,), nmax, dtype=torch.int32, device=dev) if ns is None else _as_device(ns, torch.int32, dev)
    if not isinstance(u, torch.Tensor):
        u = torch.as_tensor(np.asarray(u, dtype=np.float64))
    u = u.to(device=dev, dtype=torch.float64)
    if single and u.ndim == 1:
        u = u.unsqueeze(0)
    if u.ndim != 2 or u.shape[0] != batch or u.shape[1] < 1:
        raise ValueError(f"u must have shape [batch={batch}, nsamples]")
    u = u.contiguous()
    nsamples = u.shape[1]
    L = _lib.lib()
    nbytes = L.qubo_logz_sample_workspace_size(batch, nmax)
    if nbytes == 0:
        raise ValueError(f"unsupported sizes batch={batch}, nmax={nmax}")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    masks = torch.empty((batch, nsamples), dtype=torch.int64, device=dev)
    lz = torch.empty(batch, dtype=torch.float64, device=dev)
    status = torch.empty(batch, dtype=torch.int32, device=dev)
    with torch.cuda.device(dev):
        _lib.check(L.qubo_logz_sample(batch, Q.data_ptr(), nmax, nsd.data_ptr(), beta.data_ptr(), nsamples,
                                      u.data_ptr(), masks.data_ptr(), lz.data_ptr(), status.data_ptr(),
                                      ws.data_ptr(), nbytes, _stream(dev)))
    _raise_status(status)
    if single:
        return masks[0], lz[0]
    return masks, lz
