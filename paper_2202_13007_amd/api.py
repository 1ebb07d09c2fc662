"""Python face of libblaz: argument marshalling only.

torch provides device memory and the current stream; every step runs in the
HIP kernels behind the C ABI.  All functions take and return tensors on the
current HIP device and enqueue on ``torch.cuda.current_stream()`` without
synchronizing.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import torch

from . import _lib
from ._lib import BlazMatrixC, check

NKEPT = 28


def _stream_dev():
    """The current stream (as a C pointer) and the index of its device: the
    library enqueues there, so every tensor must live on that device."""
    st = torch.cuda.current_stream()
    return ctypes.c_void_p(st.cuda_stream), st.device_index


def _ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def code_stride(lines: int = 2) -> int:
    """Bytes of codes per block with L kept lines (28 for the paper's L = 2)."""
    v = int(_lib.lib().blaz_code_stride(lines))
    if v < 0:
        raise _lib.BlazError(v, f"code_stride({lines})")
    return v


@dataclass
class BlazMatrix:
    """A compressed rows x cols matrix on the device (45 bytes per 8x8 block).

    f, s: float64 [nblk]; phi: uint8 [nblk]; codes: int8 [nblk, code_stride(lines)]
    (28 for the paper's scheme).  Block (I, J) is entry I*(cols/8) + J.
    lines: kept lines L of DCT coefficients, the tunable rate (2: the paper's).
    """
    rows: int
    cols: int
    f: torch.Tensor
    s: torch.Tensor
    phi: torch.Tensor
    codes: torch.Tensor
    lines: int = 2
    _desc: object = field(default=None, init=False, repr=False, compare=False)

    def __setattr__(self, name, value):
        # a reassigned field invalidates the checked descriptor
        if name != "_desc":
            object.__setattr__(self, "_desc", None)
        object.__setattr__(self, name, value)

    @property
    def nblk(self) -> int:
        return (self.rows // 8) * (self.cols // 8)

    @property
    def nbytes(self) -> int:
        return self.f.nbytes + self.s.nbytes + self.phi.nbytes + self.codes.nbytes

    @staticmethod
    def empty(rows: int, cols: int, device=None, lines: int = 2) -> "BlazMatrix":
        n = _lib.lib().blaz_block_count(rows, cols)
        if n < 0:
            raise _lib.BlazError(int(n), f"BlazMatrix.empty({rows}, {cols})")
        dev = torch.device("cuda") if device is None else torch.device(device)
        return BlazMatrix(rows, cols,
                          torch.empty(n, dtype=torch.float64, device=dev),
                          torch.empty(n, dtype=torch.float64, device=dev),
                          torch.empty(n, dtype=torch.uint8, device=dev),
                          torch.empty((n, code_stride(lines)), dtype=torch.int8, device=dev), lines)

    def c(self, dev: int | None = None) -> BlazMatrixC:
        """The C descriptor, after checking that the four arrays are
        contiguous CUDA tensors on device ``dev`` (default: the current one)
        holding at least nblk records: the library sees only pointers and the
        shape.  The checked descriptor is kept until a field is reassigned
        (the arrays must not be resized in place meanwhile)."""
        if dev is None:
            dev = torch.cuda.current_device()
        d = self._desc
        if d is not None and d[0] == dev:
            return d[1]
        n = self.nblk
        _check_tensor(self.f, "BlazMatrix.f", torch.float64, n, dev)
        _check_tensor(self.s, "BlazMatrix.s", torch.float64, n, dev)
        _check_tensor(self.phi, "BlazMatrix.phi", torch.uint8, n, dev)
        _check_tensor(self.codes, "BlazMatrix.codes", torch.int8, n * code_stride(self.lines), dev)
        m = BlazMatrixC(self.rows, self.cols, self.f.data_ptr(), self.s.data_ptr(),
                        self.phi.data_ptr(), self.codes.data_ptr(), self.lines)
        object.__setattr__(self, "_desc", (dev, m))
        return m

    def to_host(self):
        """(f, s, phi, codes) as numpy arrays (synchronizes)."""
        return (self.f.cpu().numpy(), self.s.cpu().numpy(), self.phi.cpu().numpy(),
                self.codes.cpu().numpy())

    @staticmethod
    def from_host(rows, cols, f, s, phi, codes, device=None, lines: int = 2) -> "BlazMatrix":
        dev = torch.device("cuda") if device is None else torch.device(device)
        return BlazMatrix(rows, cols,
                          torch.as_tensor(f, dtype=torch.float64).to(dev).contiguous(),
                          torch.as_tensor(s, dtype=torch.float64).to(dev).contiguous(),
                          torch.as_tensor(phi, dtype=torch.uint8).to(dev).contiguous(),
                          torch.as_tensor(codes, dtype=torch.int8).reshape(-1, code_stride(lines)).to(dev)
                          .contiguous(), lines)


def _on_device(t, dev: int) -> bool:
    return isinstance(t, torch.Tensor) and t.is_cuda and t.get_device() == dev


def _check_tensor(t, what: str, dtype: torch.dtype, numel: int, dev: int):
    """A contiguous CUDA tensor of ``dtype`` on device ``dev`` with at least
    ``numel`` elements: the library reads and writes that many."""
    if not _on_device(t, dev):
        raise ValueError(f"{what}: expected a CUDA tensor on device {dev}")
    if t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{what}: expected a contiguous {dtype} tensor, got {t.dtype}")
    if t.numel() < numel:
        raise ValueError(f"{what}: {t.numel()} elements, {numel} needed")


def _check_dense(A: torch.Tensor, what: str, dev: int, shape=None):
    """A 2-D float64 CUDA tensor on device ``dev`` with unit column stride
    (rows may be strided), of exactly ``shape`` when given."""
    if not _on_device(A, dev) or A.dtype != torch.float64 or A.dim() != 2 or A.stride(1) != 1:
        raise ValueError(f"{what}: expected a 2-D float64 CUDA tensor on device {dev} with unit column stride")
    if shape is not None and tuple(A.shape) != tuple(shape):
        raise ValueError(f"{what}: shape {tuple(A.shape)}, expected {tuple(shape)}")


def _check_index(t, what: str, count: int, dev: int):
    _check_tensor(t, what, torch.int64, count, dev)
    if t.numel() != count:
        raise ValueError(f"{what}: {t.numel()} indices, expected {count}")


def compress(A: torch.Tensor, out: BlazMatrix | None = None, prec: str = "fp64",
             psi: torch.Tensor | None = None, lines: int = 2) -> BlazMatrix:
    """Compress a float64 matrix (rows, cols multiples of 8); ``lines`` sets
    the rate of a new output (ignored when ``out`` is given)."""
    stream, dev = _stream_dev()
    _check_dense(A, "compress", dev)
    rows, cols = A.shape
    if out is None:
        out = BlazMatrix.empty(rows, cols, A.device, lines)
    elif (out.rows, out.cols) != (rows, cols):
        raise ValueError(f"compress: out is {out.rows} x {out.cols}, A is {rows} x {cols}")
    if psi is not None:
        _check_tensor(psi, "compress psi", torch.uint8, 64 * out.nblk, dev)
    m = out.c(dev)
    check(_lib.lib().blaz_compress(_ptr(A), A.stride(0), ctypes.byref(m), _lib.PREC[prec], _ptr(psi),
                                   stream), "blaz_compress")
    return out


def compress_predicted(A: torch.Tensor, out: BlazMatrix | None = None,
                       psi: torch.Tensor | None = None) -> BlazMatrix:
    """Compression whose DCT takes the predicted slopes of Eq. eqpredict
    instead of the normalized block (the other reading of the transform's
    input); same record format, decompressed by ``decompress``."""
    stream, dev = _stream_dev()
    _check_dense(A, "compress_predicted", dev)
    rows, cols = A.shape
    if out is None:
        out = BlazMatrix.empty(rows, cols, A.device)
    elif (out.rows, out.cols) != (rows, cols):
        raise ValueError(f"compress_predicted: out is {out.rows} x {out.cols}, A is {rows} x {cols}")
    if psi is not None:
        _check_tensor(psi, "compress_predicted psi", torch.uint8, 64 * out.nblk, dev)
    m = out.c(dev)
    check(_lib.lib().blaz_compress_predicted(_ptr(A), A.stride(0), ctypes.byref(m), _ptr(psi), stream),
          "blaz_compress_predicted")
    return out


def decompress(x: BlazMatrix, out: torch.Tensor | None = None) -> torch.Tensor:
    stream, dev = _stream_dev()
    if out is None:
        out = torch.empty((x.rows, x.cols), dtype=torch.float64, device=x.f.device)
    _check_dense(out, "decompress", dev, (x.rows, x.cols))
    m = x.c(dev)
    check(_lib.lib().blaz_decompress(ctypes.byref(m), _ptr(out), out.stride(0), stream), "blaz_decompress")
    return out


def add(x: BlazMatrix, y: BlazMatrix, out: BlazMatrix | None = None) -> BlazMatrix:
    stream, dev = _stream_dev()
    out = BlazMatrix.empty(x.rows, x.cols, x.f.device, x.lines) if out is None else out
    mx, my, mz = x.c(dev), y.c(dev), out.c(dev)
    check(_lib.lib().blaz_add(ctypes.byref(mx), ctypes.byref(my), ctypes.byref(mz), stream), "blaz_add")
    return out


def sub(x: BlazMatrix, y: BlazMatrix, out: BlazMatrix | None = None) -> BlazMatrix:
    stream, dev = _stream_dev()
    out = BlazMatrix.empty(x.rows, x.cols, x.f.device, x.lines) if out is None else out
    mx, my, mz = x.c(dev), y.c(dev), out.c(dev)
    check(_lib.lib().blaz_sub(ctypes.byref(mx), ctypes.byref(my), ctypes.byref(mz), stream), "blaz_sub")
    return out


def scale(x: BlazMatrix, c: float, out: BlazMatrix | None = None) -> BlazMatrix:
    """out = c * x; pass out=x for the in-place form."""
    stream, dev = _stream_dev()
    out = BlazMatrix.empty(x.rows, x.cols, x.f.device, x.lines) if out is None else out
    mx, mz = x.c(dev), out.c(dev)
    check(_lib.lib().blaz_scale(ctypes.byref(mx), float(c), ctypes.byref(mz), stream), "blaz_scale")
    return out


DIAGNOSE_FIELDS = ("constant_blocks", "phi_clamps", "codes_at_127", "nonfinite_records")


def diagnose(x: BlazMatrix, counters: torch.Tensor | None = None) -> torch.Tensor:
    """Data-condition counts of x (int64 [4], see DIAGNOSE_FIELDS), added to
    ``counters`` when given (zeroed otherwise)."""
    stream, dev = _stream_dev()
    if counters is None:
        counters = torch.zeros(4, dtype=torch.int64, device=x.f.device)
    _check_tensor(counters, "diagnose counters", torch.int64, 4, dev)
    m = x.c(dev)
    check(_lib.lib().blaz_diagnose(ctypes.byref(m), _ptr(counters), stream), "blaz_diagnose")
    return counters


def dot(x: BlazMatrix, xrow: torch.Tensor, y: BlazMatrix, ycol: torch.Tensor,
        out: torch.Tensor | None = None) -> torch.Tensor:
    """out[q] = <line xrow[q] of x, column ycol[q] of y> (int64 device index tensors)."""
    stream, dev = _stream_dev()
    count = xrow.numel()
    xrow, ycol = xrow.contiguous(), ycol.contiguous()
    _check_index(xrow, "dot xrow", count, dev)
    _check_index(ycol, "dot ycol", count, dev)
    out = torch.empty(count, dtype=torch.float64, device=x.f.device) if out is None else out
    _check_tensor(out, "dot out", torch.float64, count, dev)
    mx, my = x.c(dev), y.c(dev)
    check(_lib.lib().blaz_dot(ctypes.byref(mx), _ptr(xrow), ctypes.byref(my), _ptr(ycol), count, _ptr(out),
                              stream), "blaz_dot")
    return out


def _dense_vectors(v: torch.Tensor, cols: int, count: int, what: str, dev: int) -> int:
    """ldv of the vectors of a dense dot: 0 for one shared 1-D vector of at
    least ``cols`` entries, else the row stride of a [count, >= cols] matrix."""
    if not _on_device(v, dev) or v.dtype != torch.float64:
        raise ValueError(f"{what}: expected a float64 CUDA tensor on device {dev}")
    if v.dim() == 1:
        if v.stride(0) != 1 or v.numel() < cols:
            raise ValueError(f"{what}: a shared vector needs {cols} contiguous entries")
        return 0
    if v.dim() != 2 or v.stride(1) != 1 or v.shape[0] != count or v.shape[1] < cols:
        raise ValueError(f"{what}: expected [{count}, >= {cols}] with unit column stride")
    return v.stride(0)


def dot_dense(x: BlazMatrix, xrow: torch.Tensor, v: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """out[q] = <line xrow[q] of x, v[q]> (v 2-D [count, >= cols]) or with one shared 1-D v."""
    stream, dev = _stream_dev()
    count = xrow.numel()
    xrow = xrow.contiguous()
    _check_index(xrow, "dot_dense xrow", count, dev)
    ldv = _dense_vectors(v, x.cols, count, "dot_dense v", dev)
    out = torch.empty(count, dtype=torch.float64, device=x.f.device) if out is None else out
    _check_tensor(out, "dot_dense out", torch.float64, count, dev)
    mx = x.c(dev)
    check(_lib.lib().blaz_dot_dense(ctypes.byref(mx), _ptr(xrow), _ptr(v), ldv, count, _ptr(out), stream),
          "blaz_dot_dense")
    return out


def matmul_workspace_bytes(m: int, n: int, k: int, b_compressed: bool, prec: str = "fp64") -> int:
    return int(_lib.lib().blaz_matmul_workspace_bytes(m, n, k, int(b_compressed), _lib.PREC[prec]))


def _operand_b(a: BlazMatrix, b, what: str, dev: int) -> int:
    """n of the product A B: B compressed (its descriptor carries the shape
    the library checks) or a dense float64 a.cols x n tensor."""
    if isinstance(b, BlazMatrix):
        return b.cols
    _check_dense(b, what, dev)
    if b.shape[0] != a.cols:
        raise ValueError(f"{what}: {b.shape[0]} rows, A has {a.cols} columns")
    return b.shape[1]


def matmul(a: BlazMatrix, b: BlazMatrix | torch.Tensor, out: torch.Tensor | None = None, prec: str = "fp64",
           workspace: torch.Tensor | None = None, tile: int = 0) -> torch.Tensor:
    """C = A B with A compressed and B compressed or dense float64; C dense float64.

    tile: output tile of the contraction (64 or 128); 0 = the library's choice."""
    stream, dev = _stream_dev()
    compressed_b = isinstance(b, BlazMatrix)
    n = _operand_b(a, b, "matmul B", dev)
    if out is None:
        out = torch.empty((a.rows, n), dtype=torch.float64, device=a.f.device)
    _check_dense(out, "matmul out", dev, (a.rows, n))
    if workspace is None:
        need = matmul_workspace_bytes(a.rows, n, a.cols, compressed_b, prec)
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=a.f.device)
    _check_tensor(workspace, "matmul workspace", torch.uint8, 0, dev)
    ma = a.c(dev)
    mb = b.c(dev) if compressed_b else None
    check(_lib.lib().blaz_matmul_tiled(ctypes.byref(ma), ctypes.byref(mb) if compressed_b else None,
                                       None if compressed_b else _ptr(b), n, 0 if compressed_b else b.stride(0),
                                       _ptr(out), out.stride(0), _lib.PREC[prec], _ptr(workspace),
                                       workspace.numel(), int(tile), stream), "blaz_matmul")
    return out


STATIC_SCRATCH_BYTES = 256 << 20  # BLAZ_STATIC_SCRATCH_BYTES


def matmul_static(a: BlazMatrix, b: BlazMatrix | torch.Tensor, out: torch.Tensor,
                  prec: str = "fp64") -> torch.Tensor:
    """C = A B as ``matmul``, with the workspace taken from the library's
    static scratch array (no device allocation by the library or here: the
    caller passes the output).  Calls that overlap on one device race on the
    array; calls on one stream are ordered."""
    stream, dev = _stream_dev()
    compressed_b = isinstance(b, BlazMatrix)
    n = _operand_b(a, b, "matmul_static B", dev)
    _check_dense(out, "matmul_static out", dev, (a.rows, n))
    ma = a.c(dev)
    mb = b.c(dev) if compressed_b else None
    check(_lib.lib().blaz_matmul_static(ctypes.byref(ma), ctypes.byref(mb) if compressed_b else None,
                                        None if compressed_b else _ptr(b), n, 0 if compressed_b else b.stride(0),
                                        _ptr(out), out.stride(0), _lib.PREC[prec], stream), "blaz_matmul_static")
    return out


def matmul_compressed_workspace_bytes(m: int, n: int, k: int, b_compressed: bool, prec: str = "fp64") -> int:
    return int(_lib.lib().blaz_matmul_compressed_workspace_bytes(m, n, k, int(b_compressed), _lib.PREC[prec]))


def matmul_compressed(a: BlazMatrix, b: BlazMatrix | torch.Tensor, out: BlazMatrix | None = None,
                      prec: str = "fp64", workspace: torch.Tensor | None = None, tile: int = 0) -> BlazMatrix:
    """C = A B compressed (the compression of ``matmul(a, b, prec=prec)``)."""
    stream, dev = _stream_dev()
    compressed_b = isinstance(b, BlazMatrix)
    n = _operand_b(a, b, "matmul_compressed B", dev)
    if out is None:
        out = BlazMatrix.empty(a.rows, n, a.f.device)
    if workspace is None:
        need = matmul_compressed_workspace_bytes(a.rows, n, a.cols, compressed_b, prec)
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=a.f.device)
    _check_tensor(workspace, "matmul_compressed workspace", torch.uint8, 0, dev)
    ma, mc = a.c(dev), out.c(dev)
    mb = b.c(dev) if compressed_b else None
    check(_lib.lib().blaz_matmul_compressed(ctypes.byref(ma), ctypes.byref(mb) if compressed_b else None,
                                            None if compressed_b else _ptr(b), n,
                                            0 if compressed_b else b.stride(0), ctypes.byref(mc),
                                            _lib.PREC[prec], _ptr(workspace), workspace.numel(), int(tile),
                                            stream), "blaz_matmul_compressed")
    return out


# ---------------------------------------------------------------------------
# Batching: many operations in one persistent launch
# ---------------------------------------------------------------------------

class Batch:
    """Collects operations; ``plan()`` validates them and uploads the plan.

    Items run concurrently: no item may use another item's output.  Tensors
    referenced by the items are kept alive by the batch and its plans; they
    must live on the device that is current when they are added, the device
    the plan is run on."""

    def __init__(self):
        self.items = []
        self._keep = []

    def _add(self, op, x=None, y=None, z=None, dense=None, ld=0, c=0.0, xrow=None, ycol=None, count=0, out=None):
        it = _lib.BatchItemC()
        it.op = _lib.OPS[op]
        it.reserved = 0
        empty = BlazMatrixC(0, 0, None, None, None, None)
        dev = torch.cuda.current_device()
        it.x = x.c(dev) if x is not None else empty
        it.y = y.c(dev) if y is not None else empty
        it.z = z.c(dev) if z is not None else empty
        it.dense = None if dense is None else dense.data_ptr()
        it.ld = ld
        it.c = float(c)
        it.xrow = None if xrow is None else xrow.data_ptr()
        it.ycol = None if ycol is None else ycol.data_ptr()
        it.count = count
        it.out = None if out is None else out.data_ptr()
        self.items.append(it)
        self._keep.extend(t for t in (x, y, z, dense, xrow, ycol, out) if t is not None)
        return self

    def compress(self, A: torch.Tensor, out: BlazMatrix):
        _check_dense(A, "batch compress", torch.cuda.current_device(), (out.rows, out.cols))
        return self._add("compress", x=out, dense=A, ld=A.stride(0))

    def decompress(self, x: BlazMatrix, out: torch.Tensor):
        _check_dense(out, "batch decompress", torch.cuda.current_device(), (x.rows, x.cols))
        return self._add("decompress", x=x, dense=out, ld=out.stride(0))

    def add(self, x: BlazMatrix, y: BlazMatrix, out: BlazMatrix):
        return self._add("add", x=x, y=y, z=out)

    def sub(self, x: BlazMatrix, y: BlazMatrix, out: BlazMatrix):
        return self._add("sub", x=x, y=y, z=out)

    def scale(self, x: BlazMatrix, c: float, out: BlazMatrix):
        return self._add("scale", x=x, z=out, c=c)

    def dot(self, x: BlazMatrix, xrow: torch.Tensor, y: BlazMatrix, ycol: torch.Tensor, out: torch.Tensor):
        count, dev = xrow.numel(), torch.cuda.current_device()
        _check_index(xrow, "batch dot xrow", count, dev)
        _check_index(ycol, "batch dot ycol", count, dev)
        _check_tensor(out, "batch dot out", torch.float64, count, dev)
        return self._add("dot", x=x, y=y, xrow=xrow, ycol=ycol, count=count, out=out)

    def dot_dense(self, x: BlazMatrix, xrow: torch.Tensor, v: torch.Tensor, out: torch.Tensor):
        count, dev = xrow.numel(), torch.cuda.current_device()
        _check_index(xrow, "batch dot_dense xrow", count, dev)
        ld = _dense_vectors(v, x.cols, count, "batch dot_dense v", dev)
        _check_tensor(out, "batch dot_dense out", torch.float64, count, dev)
        return self._add("dot_dense", x=x, dense=v, ld=ld, xrow=xrow, count=count, out=out)

    def _plan_into(self, host_ptr: int, nbytes: int):
        """Write the plan image into host memory; returns (n_plan, total_chunks)."""
        n = len(self.items)
        arr = (_lib.BatchItemC * max(n, 1))(*self.items)
        n_plan = ctypes.c_int64()
        total = ctypes.c_int64()
        st = _lib.lib().blaz_batch_plan(ctypes.cast(arr, ctypes.c_void_p), n, ctypes.c_void_p(host_ptr), nbytes,
                                        ctypes.byref(n_plan), ctypes.byref(total))
        if st != _lib.BLAZ_OK:
            raise _lib.BlazError(st, f"blaz_batch_plan (item {n_plan.value})")
        return n_plan.value, total.value

    def plan(self, device=None) -> "BatchPlan":
        nbytes = int(_lib.lib().blaz_batch_plan_bytes(len(self.items)))
        host = torch.empty(max(nbytes, 8), dtype=torch.uint8, pin_memory=torch.cuda.is_available())
        n_plan, total = self._plan_into(host.data_ptr(), host.numel())
        dev = torch.device("cuda") if device is None else torch.device(device)
        plan_dev = host.to(dev, non_blocking=True)
        counter = torch.zeros(1, dtype=torch.int64, device=dev)
        return BatchPlan(plan_dev, host, n_plan, total, counter, list(self._keep))


class MatmulGroup:
    """Collects binary64 products C = A B (A compressed, B compressed or
    dense float64); ``plan()`` validates them, allocates the workspace for
    the rebuilt operands and uploads the plan.  Products run concurrently:
    none may write another's operands or output."""

    def __init__(self):
        self.items = []
        self._keep = []

    def add(self, a: BlazMatrix, b: BlazMatrix | torch.Tensor, out: torch.Tensor, tile: int = 0):
        dev = torch.cuda.current_device()
        compressed_b = isinstance(b, BlazMatrix)
        n = _operand_b(a, b, "group matmul B", dev)
        _check_dense(out, "group matmul out", dev, (a.rows, n))
        it = _lib.MatmulItemC()
        it.a = a.c(dev)
        it.b = b.c(dev) if compressed_b else BlazMatrixC(0, 0, None, None, None, None)
        it.bdense = None if compressed_b else b.data_ptr()
        it.n = n
        it.ldb = 0 if compressed_b else b.stride(0)
        it.c = out.data_ptr()
        it.ldc = out.stride(0)
        it.tile = int(tile)
        it.reserved = 0
        self.items.append(it)
        self._keep.extend((a, b, out))
        return self

    def plan(self, device=None, workspace: torch.Tensor | None = None) -> "MatmulGroupPlan":
        n = len(self.items)
        arr = (_lib.MatmulItemC * max(n, 1))(*self.items)
        nbytes = int(_lib.lib().blaz_matmul_group_plan_bytes(n))
        host = torch.empty(max(nbytes, 8), dtype=torch.uint8, pin_memory=torch.cuda.is_available())
        info = _lib.MatmulGroupInfoC()
        dev = torch.device("cuda") if device is None else torch.device(device)

        def call(ws):
            return _lib.lib().blaz_matmul_group_plan(ctypes.cast(arr, ctypes.c_void_p), n,
                                                     None if ws is None else _ptr(ws),
                                                     0 if ws is None else ws.numel(),
                                                     ctypes.c_void_p(host.data_ptr()), host.numel(),
                                                     ctypes.byref(info))
        st = call(workspace)
        if st == -7 and workspace is None:  # BLAZ_ERR_WORKSPACE: size it, then plan again
            workspace = torch.empty(max(int(info.workspace_bytes), 1), dtype=torch.uint8, device=dev)
            st = call(workspace)
        if st != _lib.BLAZ_OK:
            raise _lib.BlazError(st, f"blaz_matmul_group_plan (product {info.rebuild_jobs})")
        plan_dev = host.to(dev, non_blocking=True)
        return MatmulGroupPlan(plan_dev, host, info, workspace, list(self._keep))


class MatmulGroupPlan:
    """A validated group of products resident on the device; ``run()``
    enqueues the rebuild and contraction launches."""

    def __init__(self, plan_dev, plan_host, info, workspace, keep):
        self.plan_dev, self.plan_host, self.info = plan_dev, plan_host, info
        self.workspace = workspace
        self._keep = keep

    def run(self):
        stream, dev = _stream_dev()
        if not _on_device(self.plan_dev, dev):
            raise ValueError(f"MatmulGroupPlan.run: the plan lives on {self.plan_dev.device}, the current stream "
                             f"on device {dev}")
        check(_lib.lib().blaz_matmul_group_run(_ptr(self.plan_dev), ctypes.byref(self.info), stream),
              "blaz_matmul_group_run")


class BatchPlan:
    """A validated batch resident on the device; ``run()`` enqueues it."""

    def __init__(self, plan_dev, plan_host, n_plan, total_chunks, counter, keep):
        self.plan_dev, self.plan_host = plan_dev, plan_host
        self.n_plan, self.total_chunks = n_plan, total_chunks
        self.counter = counter
        self._keep = keep

    def run(self, workgroups: int = 0, chunks_per_claim: int = 0):
        stream, dev = _stream_dev()
        if not _on_device(self.plan_dev, dev):
            raise ValueError(f"BatchPlan.run: the plan lives on {self.plan_dev.device}, the current stream on "
                             f"device {dev}")
        check(_lib.lib().blaz_batch_run(_ptr(self.plan_dev), self.n_plan, self.total_chunks, _ptr(self.counter),
                                        int(workgroups), int(chunks_per_claim), stream), "blaz_batch_run")


class ResidentBatch:
    """A plan buffer of ``capacity`` items, its run state and a pinned host
    staging area, for running successive batches through one captured HIP
    graph (``blaz_batch_run_resident``).  ``load(batch)`` plans the batch into
    the staging area and enqueues one copy of the counts and the plan image on
    the current stream; ``run()``, or a replay of ``graph(...)`` on the same
    stream, executes the plan loaded last.  Loads and runs on one stream are
    ordered, so a load never overwrites a plan under an earlier run; a load
    on another stream must wait for the earlier runs.  ``load`` waits until
    the previous load's copy has executed before it rewrites the staging
    area, which on one stream means until the earlier runs are done: rotate
    several objects to keep the host from waiting."""

    STATE_BYTES = ctypes.sizeof(_lib.BatchStateC)

    def __init__(self, capacity: int, device=None):
        if capacity < 1:
            raise ValueError("ResidentBatch: capacity must be at least 1")
        self.capacity = int(capacity)
        self.plan_bytes = int(_lib.lib().blaz_batch_plan_bytes(self.capacity))
        dev = torch.device("cuda") if device is None else torch.device(device)
        total = self.STATE_BYTES + self.plan_bytes
        self.host = torch.zeros(total, dtype=torch.uint8, pin_memory=True)
        self.dev = torch.zeros(total, dtype=torch.uint8, device=dev)
        self.state = self.dev[:self.STATE_BYTES]
        self.plan_dev = self.dev[self.STATE_BYTES:]
        self._state_host = _lib.BatchStateC.from_address(self.host.data_ptr())
        self._item_bytes = self.plan_bytes // self.capacity
        self._copied = torch.cuda.Event()
        self._loaded = False
        self._graphs = {}
        self._keep = []
        self.n_plan = self.total_chunks = 0

    def load(self, batch: Batch):
        """Plan `batch` and enqueue the copy of its counts and plan image;
        returns (n_plan, total_chunks)."""
        if len(batch.items) > self.capacity:
            raise ValueError(f"ResidentBatch.load: {len(batch.items)} items, capacity {self.capacity}")
        if self._loaded:
            self._copied.synchronize()
        n_plan, total = batch._plan_into(self.host.data_ptr() + self.STATE_BYTES, self.plan_bytes)
        st = self._state_host
        st.n_plan, st.total_chunks, st.counter, st.status = n_plan, total, 0, 0
        used = self.STATE_BYTES + n_plan * self._item_bytes
        self.dev[:used].copy_(self.host[:used], non_blocking=True)
        self._copied.record()
        self._loaded = True
        self._keep = list(batch._keep)
        self.n_plan, self.total_chunks = n_plan, total
        return n_plan, total

    def run(self, workgroups: int = 0, chunks_per_claim: int = 0):
        stream, dev = _stream_dev()
        if not _on_device(self.dev, dev):
            raise ValueError(f"ResidentBatch.run: the buffers live on {self.dev.device}, the current stream on "
                             f"device {dev}")
        check(_lib.lib().blaz_batch_run_resident(_ptr(self.plan_dev), self.capacity, _ptr(self.state),
                                                 int(workgroups), int(chunks_per_claim), stream),
              "blaz_batch_run_resident")

    def graph(self, workgroups: int = 0, chunks_per_claim: int = 0) -> "torch.cuda.CUDAGraph":
        """The run captured once per launch shape; replay it on the stream the
        loads are enqueued on (or one ordered after it)."""
        key = (int(workgroups), int(chunks_per_claim))
        g = self._graphs.get(key)
        if g is None:
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                self.run(*key)
            self._graphs[key] = g
        return g

    def status(self) -> int:
        """The status the last executed run wrote (synchronizes)."""
        return int(self.state.view(torch.int64)[3].item())
