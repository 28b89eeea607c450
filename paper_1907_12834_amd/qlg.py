"""ctypes binding of libqlg (include/qlg.h).

This module only marshals arguments: every step of the QLG path runs in the
HIP kernels of libqlg.so.  PyTorch provides device memory and the stream.
There is no CPU fallback; if the library is missing the import fails.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqlg.so")

QLG_OK = 0
STATUS_NAMES = {0: "QLG_OK", 1: "QLG_ERR_ARG", 2: "QLG_ERR_SHAPE", 3: "QLG_ERR_DTYPE",
                4: "QLG_ERR_DEVICE", 5: "QLG_ERR_OOM", 6: "QLG_ERR_STATE", 7: "QLG_ERR_NUMERIC"}
C64, C128 = 0, 1
INTERLEAVED, PLAIN = 0, 1
RECORD_DOUBLES = 16   # QLG_RECORD_DOUBLES
STATIC_SCRATCH_BYTES = 16 << 20   # QLG_STATIC_SCRATCH_BYTES

# every symbol declared in include/qlg.h
EXPORTED = [
    "qlg_version", "qlg_query_sizes", "qlg_init", "qlg_init_static", "qlg_set_psi", "qlg_get_psi", "qlg_set_qubits",
    "qlg_get_qubits", "qlg_set_potential", "qlg_fields", "qlg_vorticity", "qlg_find_vortices", "qlg_step", "qlg_observables", "qlg_record_observables", "qlg_decode_records",
    "qlg_set_tuning", "qlg_get_tuning",
    "qlg_autotune", "qlg_set_timing", "qlg_last_kernel_ms", "qlg_adjoint_query",
    "qlg_forward_record", "qlg_objective_grad", "qlg_adjoint_step", "qlg_set_psi_adjoint",
    "qlg_inject_device_error", "qlg_status_string", "qlg_last_error", "qlg_destroy",
]


class Params(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("dtype", ctypes.c_int32), ("split", ctypes.c_int32),
                ("nbatch", ctypes.c_int32), ("nx", ctypes.POINTER(ctypes.c_int64)),
                ("ny", ctypes.POINTER(ctypes.c_int64)), ("nz", ctypes.POINTER(ctypes.c_int64)),
                ("g0", ctypes.c_double),
                ("g1", ctypes.c_double), ("g2", ctypes.c_double), ("eps", ctypes.c_double)]


class Obs(ctypes.Structure):
    _fields_ = [("norm_q", ctypes.c_double), ("norm_psi", ctypes.c_double),
                ("pop", ctypes.c_double * 5), ("energy", ctypes.c_double),
                ("overlap_re", ctypes.c_double), ("overlap_im", ctypes.c_double),
                ("e_overlap_re", ctypes.c_double), ("e_overlap_im", ctypes.c_double),
                ("step", ctypes.c_int64), ("has_overlap", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self) -> dict:
        d = {"norm_q": self.norm_q, "norm_psi": self.norm_psi, "pop": list(self.pop),
             "energy": self.energy, "step": int(self.step)}
        if self.has_overlap:
            d["overlap"] = complex(self.overlap_re, self.overlap_im)
            d["e_overlap"] = complex(self.e_overlap_re, self.e_overlap_im)
        return d


class Tuning(ctypes.Structure):
    _fields_ = [("steps_per_pass", ctypes.c_int32), ("tile_rows", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("qubit_split", ctypes.c_int32)]


class QLGError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        super().__init__("%s failed with %s%s" % (where, STATUS_NAMES.get(status, status),
                                                 (": " + detail) if detail else ""))


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError("libqlg.so is not built (%s); run __graft_entry__.build() or "
                          "python -m paper_1907_12834_amd.build" % path)
    lib = ctypes.CDLL(path)
    P, vp, sz = ctypes.POINTER, ctypes.c_void_p, ctypes.c_size_t
    i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "qlg_version": (i32, []),
        "qlg_query_sizes": (i32, [P(Params), P(sz), P(sz)]),
        "qlg_init": (i32, [P(Params), vp, sz, vp, sz, vp, P(vp)]),
        "qlg_init_static": (i32, [P(Params), vp, sz, vp, P(vp)]),
        "qlg_set_psi": (i32, [vp, vp]),
        "qlg_get_psi": (i32, [vp, vp]),
        "qlg_set_qubits": (i32, [vp, vp]),
        "qlg_get_qubits": (i32, [vp, vp]),
        "qlg_set_potential": (i32, [vp, vp, dbl]),
        "qlg_fields": (i32, [vp, vp, vp, vp, vp]),
        "qlg_vorticity": (i32, [vp, i32, vp, vp]),
        "qlg_find_vortices": (i32, [vp, i32, vp, vp, i64, vp]),
        "qlg_step": (i32, [vp, i64]),
        "qlg_observables": (i32, [vp, P(Obs)]),
        "qlg_record_observables": (i32, [vp, vp]),
        "qlg_decode_records": (i32, [vp, vp, i64, P(Obs)]),
        "qlg_set_tuning": (i32, [vp, P(Tuning)]),
        "qlg_get_tuning": (i32, [vp, P(Tuning)]),
        "qlg_autotune": (i32, [vp]),
        "qlg_set_timing": (i32, [vp, i32]),
        "qlg_last_kernel_ms": (i32, [vp, P(dbl), P(i64)]),
        "qlg_adjoint_query": (i32, [P(Params), i64, i32, P(sz), P(sz)]),
        "qlg_forward_record": (i32, [vp, i64, i32, vp, sz]),
        "qlg_objective_grad": (i32, [vp, i32, vp, vp, P(dbl), P(dbl)]),
        "qlg_adjoint_step": (i32, [vp, i64, i32, vp, vp, vp, sz, P(dbl)]),
        "qlg_set_psi_adjoint": (i32, [vp, vp, vp]),
        "qlg_inject_device_error": (i32, [vp, ctypes.c_char_p]),
        "qlg_status_string": (ctypes.c_char_p, [i32]),
        "qlg_last_error": (ctypes.c_char_p, [vp]),
        "qlg_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_LIB: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load_library()
    return _LIB


def make_params(ndim: int, nx: Sequence[int], ny: Optional[Sequence[int]], g, eps: float,
                dtype: int = C128, split: int = INTERLEAVED, nz: Optional[Sequence[int]] = None):
    nb = len(nx)
    P64 = ctypes.POINTER(ctypes.c_int64)
    nx_arr = (ctypes.c_int64 * nb)(*[int(v) for v in nx])
    ny_arr = (ctypes.c_int64 * nb)(*[int(v) for v in ny]) if ny is not None else None
    nz_arr = (ctypes.c_int64 * nb)(*[int(v) for v in nz]) if nz is not None else None
    p = Params(ndim, dtype, split, nb, nx_arr,
               ctypes.cast(ny_arr, P64) if ny_arr is not None else None,
               ctypes.cast(nz_arr, P64) if nz_arr is not None else None,
               float(g[0]), float(g[1]), float(g[2]), float(eps))
    return p, (nx_arr, ny_arr, nz_arr)


def query_sizes(params: Params):
    s, c = ctypes.c_size_t(), ctypes.c_size_t()
    st = lib().qlg_query_sizes(ctypes.byref(params), ctypes.byref(s), ctypes.byref(c))
    if st != QLG_OK:
        raise QLGError(st, "qlg_query_sizes")
    return s.value, c.value


def _device_bytes(nbytes: int, device) -> torch.Tensor:
    # 256-byte alignment is guaranteed by the caching allocator
    t = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)
    assert t.data_ptr() % 256 == 0
    return t


class Lattice:
    """One context over caller-owned (torch) device buffers.

    ``psi`` arguments use the canonical layout: a complex tensor per instance
    of shape (5, nx) in 1D, (5, ny, nx) in 2D or (5, nz, ny, nx) in 3D,
    components ordered m = 2..-2; batches are passed as lists.
    """

    def __init__(self, ndim: int, nx: Sequence[int], ny: Optional[Sequence[int]] = None,
                 nz: Optional[Sequence[int]] = None,
                 g=(1.0, -0.5, 0.5), eps: float = 0.1, dtype: str = "c128",
                 split: str = "interleaved", device="cuda:0", stream: Optional[torch.cuda.Stream] = None,
                 static_scratch: bool = False):
        if not torch.cuda.is_available():
            raise RuntimeError("libqlg needs a HIP device; none is visible")
        self.ndim = ndim
        self.nx = [int(v) for v in nx]
        self.ny = [int(v) for v in ny] if ny is not None else [1] * len(self.nx)
        self.nz = [int(v) for v in nz] if nz is not None else [1] * len(self.nx)
        self.g = tuple(float(v) for v in g)
        self.eps = float(eps)
        self.dtype_code = {"c64": C64, "c128": C128}[dtype]
        self.torch_dtype = torch.complex64 if self.dtype_code == C64 else torch.complex128
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.params, self._keep = make_params(ndim, self.nx, ny if ndim >= 2 else None, self.g, self.eps,
                                              self.dtype_code,
                                              {"interleaved": INTERLEAVED, "plain": PLAIN}[split],
                                              nz if ndim == 3 else None)
        sb, cb = query_sizes(self.params)
        self.state_buf = _device_bytes(sb, self.device)
        self._pot = None   # device copy of the external potential while one is set
        ctx = ctypes.c_void_p()
        if static_scratch:
            # the library's per-GPU scratch array (qlg_init_static): no scratch buffer here
            self.scratch_buf = None
            with torch.cuda.device(self.device):
                st = lib().qlg_init_static(ctypes.byref(self.params), self.state_buf.data_ptr(), sb,
                                           ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx))
            if st != QLG_OK:
                raise QLGError(st, "qlg_init_static")
        else:
            self.scratch_buf = _device_bytes(cb, self.device)
            st = lib().qlg_init(ctypes.byref(self.params), self.state_buf.data_ptr(), sb,
                                self.scratch_buf.data_ptr(), cb, ctypes.c_void_p(self.stream.cuda_stream),
                                ctypes.byref(ctx))
            if st != QLG_OK:
                raise QLGError(st, "qlg_init")
        self.ctx = ctx

    # -- helpers -------------------------------------------------------------
    @property
    def nbatch(self) -> int:
        return len(self.nx)

    @property
    def sites(self) -> int:
        return int(sum(a * b * c for a, b, c in zip(self.nx, self.ny, self.nz)))

    def _check(self, st: int, where: str):
        if st != QLG_OK:
            msg = lib().qlg_last_error(self.ctx)
            raise QLGError(st, where, msg.decode() if msg else "")

    def _shape(self, i: int):
        return (5, self.nx[i]) if self.ndim == 1 else (5, self.ny[i], self.nx[i]) if self.ndim == 2 \
            else (5, self.nz[i], self.ny[i], self.nx[i])

    def _flat(self, fields: List, per_site: int) -> torch.Tensor:
        parts = []
        for i, f in enumerate(fields):
            t = torch.as_tensor(f) if not isinstance(f, torch.Tensor) else f
            t = t.to(device=self.device, dtype=self.torch_dtype)
            n = per_site * self.nx[i] * self.ny[i] * self.nz[i]
            if t.numel() != n:
                raise ValueError("field %d has %d elements, expected %d" % (i, t.numel(), n))
            parts.append(t.reshape(-1))
        return torch.cat(parts).contiguous()

    def _unflat(self, flat: torch.Tensor, per_site: int):
        out, o = [], 0
        for i in range(self.nbatch):
            n = per_site * self.nx[i] * self.ny[i] * self.nz[i]
            shape = self._shape(i)
            shape = shape if per_site == 5 else (2,) + shape
            out.append(flat[o:o + n].reshape(shape))
            o += n
        return out

    # -- API -----------------------------------------------------------------
    def set_psi(self, psi):
        fields = psi if isinstance(psi, (list, tuple)) else [psi]
        self._psi_in = self._flat(fields, 5)
        self._check(lib().qlg_set_psi(self.ctx, self._psi_in.data_ptr()), "qlg_set_psi")

    def get_psi(self) -> List[torch.Tensor]:
        flat = torch.empty(5 * self.sites, dtype=self.torch_dtype, device=self.device)
        self._check(lib().qlg_get_psi(self.ctx, flat.data_ptr()), "qlg_get_psi")
        return self._unflat(flat, 5)

    def set_qubits(self, qubits):
        """qubits: per instance a tensor (2, 5, ...) = (a, b)."""
        fields = qubits if isinstance(qubits, (list, tuple)) else [qubits]
        self._qb_in = self._flat(fields, 10)
        self._check(lib().qlg_set_qubits(self.ctx, self._qb_in.data_ptr()), "qlg_set_qubits")

    def get_qubits(self) -> List[torch.Tensor]:
        flat = torch.empty(10 * self.sites, dtype=self.torch_dtype, device=self.device)
        self._check(lib().qlg_get_qubits(self.ctx, flat.data_ptr()), "qlg_get_qubits")
        return self._unflat(flat, 10)

    def set_potential(self, V=None, mu: float = 0.0):
        """External potential V(x) (per instance an array of the lattice's spatial shape, or None)
        and chemical potential mu (Sec. II "Additional terms"); set_potential() removes both.
        The device copy of V is kept by this object for as long as the library uses it."""
        if V is None:
            self._pot = None
        else:
            fields = V if isinstance(V, (list, tuple)) else [V]
            if len(fields) != self.nbatch:
                raise ValueError("need one potential per instance (%d)" % self.nbatch)
            parts = []
            for i, f in enumerate(fields):
                t = torch.as_tensor(f).to(device=self.device, dtype=torch.float64)
                if t.numel() != self.nx[i] * self.ny[i] * self.nz[i]:
                    raise ValueError("potential %d has %d values, expected %d" %
                                     (i, t.numel(), self.nx[i] * self.ny[i] * self.nz[i]))
                parts.append(t.reshape(-1))
            self._pot = torch.cat(parts).contiguous()
        self._check(lib().qlg_set_potential(self.ctx, self._pot.data_ptr() if self._pot is not None else None,
                                            float(mu)), "qlg_set_potential")

    def _unflat_scalar(self, flat: torch.Tensor) -> List[torch.Tensor]:
        out, o = [], 0
        for i in range(self.nbatch):
            n = self.nx[i] * self.ny[i] * self.nz[i]
            out.append(flat[o:o + n].reshape(self._shape(i)[1:]))
            o += n
        return out

    def fields(self, which: Sequence[str] = ("n", "f_par", "f_perp", "a00")) -> List[dict]:
        """Per instance, the FP64 fields n, F_par, F_perp, |A00| (Sec. III eq. cmap) named in `which`."""
        names = ("n", "f_par", "f_perp", "a00")
        bad = [w for w in which if w not in names]
        if bad or not which:
            raise ValueError("fields must be a non-empty subset of %s" % (names,))
        bufs = {w: torch.empty(self.sites, dtype=torch.float64, device=self.device) for w in which}
        ptrs = [bufs[w].data_ptr() if w in bufs else None for w in names]
        self._check(lib().qlg_fields(self.ctx, *ptrs), "qlg_fields")
        per = {w: self._unflat_scalar(b) for w, b in bufs.items()}
        return [{w: per[w][i] for w in which} for i in range(self.nbatch)]

    def vorticity(self, m_index: int, omega: bool = True, winding: bool = True) -> List[dict]:
        """Per instance {"omega": FP64, "winding": int32} of component m_index (Sec. VI): shape
        (ny, nx) in 2D; (3, nz, ny, nx) in 3D, the plaquettes normal to x, y and z."""
        ncomp = 3 if self.ndim == 3 else 1
        om = torch.empty(ncomp * self.sites, dtype=torch.float64, device=self.device) if omega else None
        wd = torch.empty(ncomp * self.sites, dtype=torch.int32, device=self.device) if winding else None
        self._check(lib().qlg_vorticity(self.ctx, int(m_index), om.data_ptr() if om is not None else None,
                                        wd.data_ptr() if wd is not None else None), "qlg_vorticity")
        out = [dict() for _ in range(self.nbatch)]
        for key, buf in (("omega", om), ("winding", wd)):
            if buf is None:
                continue
            parts = [self._unflat_scalar(b) for b in buf.view(ncomp, self.sites)]
            for i in range(self.nbatch):
                out[i][key] = parts[0][i] if ncomp == 1 else torch.stack([p[i] for p in parts])
        return out

    def find_vortices(self, m_index: int, capacity: int = 4096) -> torch.Tensor:
        """Vortex cores of component m_index (Sec. VI): an int32 tensor on the device, (k, 4) of
        (instance, y, x, winding) rows in (instance, y, x) order in 2D; (k, 6) of (instance,
        family, z, y, x, winding) rows in (family, instance, z, y, x) order in 3D, family 0, 1, 2
        the plaquettes normal to x, y, z."""
        ncomp, width = (3, 6) if self.ndim == 3 else (1, 4)
        wind = torch.empty(ncomp * self.sites, dtype=torch.int32, device=self.device)
        count = torch.zeros(1, dtype=torch.int64, device=self.device)
        while True:
            cores = torch.empty((max(int(capacity), 1), width), dtype=torch.int32, device=self.device)
            self._check(lib().qlg_find_vortices(self.ctx, int(m_index), wind.data_ptr(), cores.data_ptr(),
                                                int(capacity), count.data_ptr()), "qlg_find_vortices")
            n = int(count.item())
            if n <= capacity:
                return cores[:n]
            capacity = n

    def track_vortices(self, m_index: int, nsteps: int, every: int) -> List[tuple]:
        """Advance nsteps, listing the cores of component m_index every `every` steps (and at the
        start): [(step, cores on the device as find_vortices returns them), ...], the paper's
        vortex tracks."""
        out = [(0, self.find_vortices(m_index))]
        done = 0
        while done < nsteps:
            n = min(int(every), nsteps - done)
            self.step(n)
            done += n
            out.append((done, self.find_vortices(m_index)))
        return out

    def step(self, nsteps: int = 1):
        self._check(lib().qlg_step(self.ctx, int(nsteps)), "qlg_step")

    def observables(self, check: bool = True) -> List[dict]:
        arr = (Obs * self.nbatch)()
        st = lib().qlg_observables(self.ctx, arr)
        if check:
            self._check(st, "qlg_observables")
        return [o.as_dict() for o in arr]

    def new_records(self, nrec: int) -> torch.Tensor:
        """Device buffer for `nrec` observables records of every instance."""
        return torch.zeros((int(nrec), self.nbatch, RECORD_DOUBLES), dtype=torch.float64, device=self.device)

    def record_observables(self, rec: torch.Tensor, k: int = 0):
        """Enqueue the observables of the current state into record slot k of `rec` (no sync)."""
        if not (rec.is_cuda and rec.dtype == torch.float64 and rec.is_contiguous()
                and rec.dim() == 3 and rec.shape[1:] == (self.nbatch, RECORD_DOUBLES) and 0 <= k < rec.shape[0]):
            raise ValueError("rec must be a contiguous float64 device tensor (nrec, nbatch, %d)" % RECORD_DOUBLES)
        self._check(lib().qlg_record_observables(self.ctx, rec[k].data_ptr()), "qlg_record_observables")

    def decode_records(self, rec, check: bool = True) -> List[List[dict]]:
        """Records (device or host tensor (nrec, nbatch, 16)) -> per record, per instance dicts."""
        if rec.is_cuda:
            with torch.cuda.stream(self.stream):   # ordered after the kernels that wrote it
                host = rec.detach().to("cpu", torch.float64).contiguous()
        else:
            host = rec.detach().to(torch.float64).contiguous()
        nrec = host.shape[0]
        arr = (Obs * (nrec * self.nbatch))()
        st = lib().qlg_decode_records(self.ctx, host.data_ptr(), nrec, arr)
        if check:
            self._check(st, "qlg_decode_records")
        return [[arr[r * self.nbatch + i].as_dict() for i in range(self.nbatch)] for r in range(nrec)]

    def run(self, nsteps: int, every: int) -> List[List[dict]]:
        """nsteps steps with the observables recorded after every `every` steps on the device;
        one host synchronisation at the end."""
        nrec = nsteps // every
        rec = self.new_records(max(nrec, 1))
        for k in range(nrec):
            self.step(every)
            self.record_observables(rec, k)
        if nsteps - nrec * every:
            self.step(nsteps - nrec * every)
        return self.decode_records(rec[:nrec]) if nrec else []

    def tuning(self) -> dict:
        t = Tuning()
        self._check(lib().qlg_get_tuning(self.ctx, ctypes.byref(t)), "qlg_get_tuning")
        return {"steps_per_pass": t.steps_per_pass, "tile_rows": t.tile_rows, "use_graph": t.use_graph,
                "qubit_split": t.qubit_split}

    def set_tuning(self, steps_per_pass: Optional[int] = None, tile_rows: Optional[int] = None,
                   use_graph: Optional[bool] = None, qubit_split: Optional[int] = None):
        """Set the launch plan (qlg_tuning in include/qlg.h); fields left None keep their value."""
        cur = self.tuning()
        t = Tuning(steps_per_pass if steps_per_pass is not None else cur["steps_per_pass"],
                   tile_rows if tile_rows is not None else cur["tile_rows"],
                   int(use_graph) if use_graph is not None else cur["use_graph"],
                   int(qubit_split) if qubit_split is not None else cur["qubit_split"])
        self._check(lib().qlg_set_tuning(self.ctx, ctypes.byref(t)), "qlg_set_tuning")

    def autotune(self) -> dict:
        self._check(lib().qlg_autotune(self.ctx), "qlg_autotune")
        return self.tuning()

    def set_timing(self, enable: bool):
        self._check(lib().qlg_set_timing(self.ctx, int(bool(enable))), "qlg_set_timing")

    def last_kernel_ms(self):
        ms, n = ctypes.c_double(), ctypes.c_int64()
        self._check(lib().qlg_last_kernel_ms(self.ctx, ctypes.byref(ms), ctypes.byref(n)),
                    "qlg_last_kernel_ms")
        return ms.value, n.value

    # -- adjoint ---------------------------------------------------------------
    def adjoint_sizes(self, nsteps: int, checkpoint_every: int):
        ck, wk = ctypes.c_size_t(), ctypes.c_size_t()
        st = lib().qlg_adjoint_query(ctypes.byref(self.params), int(nsteps), int(checkpoint_every),
                                     ctypes.byref(ck), ctypes.byref(wk))
        if st != QLG_OK:
            raise QLGError(st, "qlg_adjoint_query")
        return ck.value, wk.value

    def forward_record(self, nsteps: int, checkpoint_every: int) -> torch.Tensor:
        """Run nsteps, keeping a checkpoint every `checkpoint_every` steps (returned buffer)."""
        ck, _ = self.adjoint_sizes(nsteps, checkpoint_every)
        buf = _device_bytes(ck, self.device)
        self._check(lib().qlg_forward_record(self.ctx, int(nsteps), int(checkpoint_every), buf.data_ptr(), ck),
                    "qlg_forward_record")
        return buf

    def objective_grad(self, kind: str = "energy", target=None):
        """(L, lambda, dL/dg explicit): lambda is complex128 in the canonical qubits layout."""
        lam = torch.empty(10 * self.sites, dtype=torch.complex128, device=self.device)
        val = ctypes.c_double()
        dg = (ctypes.c_double * 3)()
        tptr = None
        if kind == "fidelity":
            fields = target if isinstance(target, (list, tuple)) else [target]
            self._target = self._flat(fields, 5)
            tptr = self._target.data_ptr()
        code = {"energy": 0, "fidelity": 1}[kind]
        self._check(lib().qlg_objective_grad(self.ctx, code, tptr, lam.data_ptr(), ctypes.byref(val), dg),
                    "qlg_objective_grad")
        return val.value, lam, list(dg)

    def adjoint_step(self, nsteps: int, checkpoint_every: int, ckpt: torch.Tensor, lam: torch.Tensor,
                     overlap: bool = True):
        """Pull lam (complex128 canonical qubits) back over the recorded run; returns dL/dg.
        overlap=False passes the workspace without its second set of segment inputs
        (checkpoint_every x 4 ndim state copies, checkpoint_every for the plain split): less device
        memory, the segment recompute then runs on the context's stream between the sweeps."""
        ck, wk = self.adjoint_sizes(nsteps, checkpoint_every)
        if not overlap and nsteps > 0:
            copy = ck // -(-int(nsteps) // int(checkpoint_every))
            nrec = 1 if self.params.split == 1 else 4 * self.params.ndim
            wk -= (int(checkpoint_every) * nrec * copy + 255) // 256 * 256
        work = _device_bytes(wk, self.device)
        dg = (ctypes.c_double * 3)(0.0, 0.0, 0.0)
        lam = lam.contiguous()
        self._check(lib().qlg_adjoint_step(self.ctx, int(nsteps), int(checkpoint_every), ckpt.data_ptr(),
                                           lam.data_ptr(), work.data_ptr(), wk, dg), "qlg_adjoint_step")
        return list(dg)

    def set_psi_adjoint(self, lam: torch.Tensor) -> List[torch.Tensor]:
        """Cotangent of psi from that of both qubits (adjoint of set_psi's a = b = psi / 2):
        lam complex128 in the canonical qubits layout; per instance a complex128 (5, ...) tensor."""
        lam = lam.contiguous()
        if not (lam.is_cuda and lam.dtype == torch.complex128 and lam.numel() == 10 * self.sites):
            raise ValueError("lam must be a complex128 device tensor of %d elements" % (10 * self.sites))
        dpsi = torch.empty(5 * self.sites, dtype=torch.complex128, device=self.device)
        self._check(lib().qlg_set_psi_adjoint(self.ctx, lam.data_ptr(), dpsi.data_ptr()), "qlg_set_psi_adjoint")
        out, o = [], 0
        for i in range(self.nbatch):
            n = 5 * self.nx[i] * self.ny[i] * self.nz[i]
            out.append(dpsi[o:o + n].reshape(self._shape(i)))
            o += n
        return out

    def close(self):
        if getattr(self, "ctx", None):
            lib().qlg_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def to_numpy_fields(tensors: List[torch.Tensor]) -> List[np.ndarray]:
    return [t.detach().to("cpu").numpy().astype(np.complex128) for t in tensors]
