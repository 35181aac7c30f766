"""ctypes binding of libebcc.so (the C ABI in include/ebcc.h).

Argument marshalling only: every step of compression and decompression runs
in the library's HIP kernels.  Tensors are PyTorch CUDA (HIP) tensors; the
current torch stream is passed to the library.  There is no CPU fallback: if
the library is missing, loading fails with an error.
"""
import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libebcc.so")

OK, EINVAL, ENOSPC, ECORRUPT, ENOMEM, EHIP, ENOTIMPL = 0, -1, -2, -3, -4, -5, -6
BOUND_REL, BOUND_ABS = 0, 1
MODE_CONST, MODE_RAW, MODE_CODED = 0, 1, 2
HDR_BYTES = 48

SYMBOLS = ("ebcc_params_default", "ebcc_compress_bound", "ebcc_compress", "ebcc_decompress", "ebcc_stream_info",
           "ebcc_release", "ebcc_status_str", "ebcc_last_error", "ebcc_compress_trace", "ebcc_profile_enable",
           "ebcc_profile_read", "ebcc_profile_stage_name", "ebcc_compress_batch", "ebcc_decompress_batch",
           "ebcc_tuning_get", "ebcc_tuning_set", "ebcc_workspace_size", "ebcc_workspace_size_batch",
           "ebcc_workspace_reserve", "ebcc_device_bytes", "ebcc_compress_noalloc",
           "ebcc_decompress_batch_async")


class Params(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("bound_mode", C.c_uint32), ("err_bound", C.c_double),
                ("base_ratio", C.c_double), ("q", C.c_double), ("levels", C.c_uint32), ("cblk_log2w", C.c_uint32),
                ("cblk_log2h", C.c_uint32), ("spiht_tile", C.c_uint32), ("trunc", C.c_uint32),
                ("bypass", C.c_uint32)]


class Tuning(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("t1_encoder", C.c_int32), ("t1_decoder", C.c_int32),
                ("t1_wave_max", C.c_int32), ("spiht", C.c_int32), ("t1_lanes", C.c_int32),
                ("t1_split", C.c_int32), ("t1_persist", C.c_int32)]


class EbccError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


_lib = None


def lib():
    """Load libebcc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first (__graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        P, S = C.c_void_p, C.c_size_t
        L.ebcc_params_default.argtypes = [C.POINTER(Params)]
        L.ebcc_params_default.restype = None
        L.ebcc_compress_bound.argtypes = [S, S]
        L.ebcc_compress_bound.restype = S
        L.ebcc_compress.argtypes = [P, S, S, C.POINTER(Params), P, S, C.POINTER(S), P]
        L.ebcc_compress_noalloc.argtypes = [P, S, S, C.POINTER(Params), P, S, C.POINTER(S), P]
        L.ebcc_compress_trace.argtypes = [P, S, S, C.POINTER(Params), P, S, C.POINTER(S), P, P, P, P, P, P, P]
        L.ebcc_decompress.argtypes = [P, S, P, S, S, P]
        L.ebcc_compress_batch.argtypes = [C.c_int, P, P, P, P, C.POINTER(Params), P, S, P, P, P, P]
        L.ebcc_workspace_size.argtypes = [S, S, C.POINTER(Params)]
        L.ebcc_workspace_size.restype = S
        L.ebcc_workspace_size_batch.argtypes = [C.c_int, P, P, C.POINTER(Params), P, P]
        L.ebcc_workspace_size_batch.restype = S
        L.ebcc_workspace_reserve.argtypes = [S, P]
        L.ebcc_device_bytes.argtypes = []
        L.ebcc_device_bytes.restype = S
        L.ebcc_decompress_batch.argtypes = [C.c_int, P, P, P, P, P, P, P]
        L.ebcc_decompress_batch_async.argtypes = [C.c_int, P, P, P, P, P, P, C.POINTER(Params), P, P]
        L.ebcc_stream_info.argtypes = [P, S, C.POINTER(S), C.POINTER(S), C.POINTER(C.c_int)]
        L.ebcc_tuning_get.argtypes = [C.POINTER(Tuning)]
        L.ebcc_tuning_set.argtypes = [C.POINTER(Tuning)]
        L.ebcc_release.argtypes = []
        L.ebcc_release.restype = None
        L.ebcc_status_str.argtypes = [C.c_int]
        L.ebcc_status_str.restype = C.c_char_p
        L.ebcc_last_error.argtypes = []
        L.ebcc_last_error.restype = C.c_char_p
        L.ebcc_profile_enable.argtypes = [C.c_int]
        L.ebcc_profile_enable.restype = None
        L.ebcc_profile_read.argtypes = [P, P, C.c_int]
        L.ebcc_profile_stage_name.argtypes = [C.c_int]
        L.ebcc_profile_stage_name.restype = C.c_char_p
        _lib = L
    return _lib


def params(err_bound=0.01, base_ratio=30.0, bound_mode=BOUND_REL, levels=5, cblk_log2w=5, cblk_log2h=5,
           spiht_tile=1, q=0.0, trunc=0, bypass=0):
    p = Params()
    lib().ebcc_params_default(C.byref(p))
    p.err_bound, p.base_ratio, p.bound_mode = float(err_bound), float(base_ratio), int(bound_mode)
    p.levels, p.cblk_log2w, p.cblk_log2h, p.spiht_tile, p.q = levels, cblk_log2w, cblk_log2h, spiht_tile, float(q)
    p.trunc = int(trunc)
    p.bypass = int(bypass)
    return p


def _check(rc):
    if rc != OK:
        raise EbccError(rc, lib().ebcc_last_error().decode() or lib().ebcc_status_str(rc).decode())


def _stream_ptr(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev_f32(x):
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float32 and x.dim() == 2):
        raise TypeError("expected a 2-D float32 tensor on the GPU")
    return x.contiguous()


def compress_bound(ny, nx):
    return lib().ebcc_compress_bound(ny, nx)


def compress_into(x, out, p, stream=None):
    """Compress x into the uint8 device tensor `out`; returns (rc, length)."""
    n = C.c_size_t(0)
    rc = lib().ebcc_compress(C.c_void_p(x.data_ptr()), x.shape[0], x.shape[1], C.byref(p), C.c_void_p(out.data_ptr()),
                             out.numel(), C.byref(n), _stream_ptr(stream))
    return rc, n.value


def compress_noalloc_into(x, out, p, stream=None):
    """ebcc_compress_noalloc: like compress_into, with the library's static
    scratch array instead of an allocated workspace; returns (rc, length)."""
    n = C.c_size_t(0)
    rc = lib().ebcc_compress_noalloc(C.c_void_p(x.data_ptr()), x.shape[0], x.shape[1], C.byref(p),
                                     C.c_void_p(out.data_ptr()), out.numel(), C.byref(n), _stream_ptr(stream))
    return rc, n.value


def compress(x, err_bound=0.01, base_ratio=30.0, out=None, stream=None, **kw):
    """Compress a 2-D float32 CUDA tensor; returns a uint8 CUDA tensor (a view
    of `out` when given)."""
    x = _dev_f32(x)
    p = params(err_bound, base_ratio, **kw)
    if out is None:
        out = torch.empty(compress_bound(*x.shape), dtype=torch.uint8, device=x.device)
    rc, n = compress_into(x, out, p, stream)
    _check(rc)
    return out[:n]


def compress_trace(x, err_bound=0.01, base_ratio=30.0, stream=None, **kw):
    """Compress and also return intermediate results for stage comparison."""
    x = _dev_f32(x)
    p = params(err_bound, base_ratio, **kw)
    out = torch.empty(compress_bound(*x.shape), dtype=torch.uint8, device=x.device)
    coef = torch.zeros_like(x)
    abase = torch.zeros_like(x)
    cres = torch.zeros_like(x)
    nblk_cap = x.numel() + 64
    kb = torch.zeros(nblk_cap, dtype=torch.uint8, device=x.device)
    pb = torch.zeros(nblk_cap, dtype=torch.uint8, device=x.device)
    info = (C.c_int32 * 11)()
    n = C.c_size_t(0)
    rc = lib().ebcc_compress_trace(C.c_void_p(x.data_ptr()), x.shape[0], x.shape[1], C.byref(p),
                                   C.c_void_p(out.data_ptr()), out.numel(), C.byref(n), _stream_ptr(stream),
                                   C.c_void_p(coef.data_ptr()), C.c_void_p(abase.data_ptr()),
                                   C.c_void_p(cres.data_ptr()), C.c_void_p(kb.data_ptr()), C.c_void_p(pb.data_ptr()),
                                   info)
    _check(rc)
    torch.cuda.synchronize()
    f = list(info)
    nb = f[6]
    d = dict(coef=coef, abase=abase, cres=cres, kb=kb[:nb], pb=pb[:nb])
    keys = ("mode", "L", "e0", "e_r", "n_max", "n_s", "nblocks", "ntiles", "base_bytes", "resid_bytes", "checks")
    d.update(zip(keys, f))
    return out[: n.value], d


def decompress_into(stream_bytes, out, stream=None):
    return lib().ebcc_decompress(C.c_void_p(stream_bytes.data_ptr()), stream_bytes.numel(), C.c_void_p(out.data_ptr()),
                                 out.shape[0], out.shape[1], _stream_ptr(stream))


def decompress(stream_bytes, ny, nx, out=None, stream=None):
    """Decompress a uint8 CUDA tensor holding one stream into a float32
    CUDA tensor of shape (ny, nx)."""
    if not (isinstance(stream_bytes, torch.Tensor) and stream_bytes.is_cuda and stream_bytes.dtype == torch.uint8):
        raise TypeError("expected a uint8 tensor on the GPU")
    stream_bytes = stream_bytes.contiguous()
    if out is None:
        out = torch.empty((ny, nx), dtype=torch.float32, device=stream_bytes.device)
    _check(decompress_into(stream_bytes, out, stream))
    return out


def _arr(ctype, vals):
    return (ctype * max(1, len(vals)))(*vals)


class BatchArgs:
    """Host argument arrays of a batched call, built once for a fixed set of
    device tensors (so a serving loop or a timed loop marshals nothing)."""

    def __init__(self, xs, outs=None, err_bounds=None):
        self.n = len(xs)
        self.xs = xs
        self.d_x = _arr(C.c_void_p, [x.data_ptr() for x in xs])
        self.ny = _arr(C.c_size_t, [x.shape[0] for x in xs])
        self.nx = _arr(C.c_size_t, [x.shape[1] for x in xs])
        self.err = None if err_bounds is None else _arr(C.c_double, [float(e) for e in err_bounds])
        self.offsets = (C.c_uint64 * max(1, self.n))()
        self.lengths = (C.c_uint64 * max(1, self.n))()
        self.status = (C.c_int * max(1, self.n))()

    def bound(self):
        return sum(compress_bound(x.shape[0], x.shape[1]) for x in self.xs)


def compress_batch_into(args, out, p, stream=None):
    """Compress args.xs into `out` (uint8 device tensor); returns rc.  Offsets,
    lengths and per-field statuses are left in args.offsets / args.lengths /
    args.status."""
    return lib().ebcc_compress_batch(args.n, args.d_x, args.ny, args.nx, args.err, C.byref(p),
                                     C.c_void_p(out.data_ptr()), out.numel(), args.offsets, args.lengths,
                                     args.status, _stream_ptr(stream))


def compress_batch(xs, err_bounds=None, err_bound=0.01, base_ratio=30.0, stream=None, check=True, **kw):
    """Compress a list of 2-D float32 CUDA tensors in one batched call;
    returns a list of uint8 CUDA tensors (views of one buffer).  With
    check=False returns (streams, statuses) instead of raising on the first
    bad field (a failed field's stream is None)."""
    xs = [_dev_f32(x) for x in xs]
    args = BatchArgs(xs, err_bounds=err_bounds)
    p = params(err_bound, base_ratio, **kw)
    dev = xs[0].device if xs else torch.device("cuda")
    out = torch.empty(max(1, args.bound()), dtype=torch.uint8, device=dev)
    rc = compress_batch_into(args, out, p, stream)
    if check:
        _check(rc)
    st = [args.status[i] for i in range(args.n)]
    streams = [out[args.offsets[i]: args.offsets[i] + args.lengths[i]] if st[i] == OK else None
               for i in range(args.n)]
    return streams if check else (streams, st)


class DecodeArgs:
    """Host argument arrays of a batched decompression (streams -> outputs)."""

    def __init__(self, streams, outs):
        self.n = len(streams)
        self.keep = (streams, outs)
        self.d_in = _arr(C.c_void_p, [s.data_ptr() for s in streams])
        self.in_len = _arr(C.c_size_t, [s.numel() for s in streams])
        self.d_x = _arr(C.c_void_p, [o.data_ptr() for o in outs])
        self.ny = _arr(C.c_size_t, [o.shape[0] for o in outs])
        self.nx = _arr(C.c_size_t, [o.shape[1] for o in outs])
        self.status = (C.c_int * max(1, self.n))()


def decompress_batch_into(args, stream=None):
    """Decompress; returns rc (per-stream statuses in args.status)."""
    return lib().ebcc_decompress_batch(args.n, args.d_in, args.in_len, args.d_x, args.ny, args.nx, args.status,
                                       _stream_ptr(stream))


def decompress_batch(streams, shapes, stream=None, check=True):
    """Decompress a list of uint8 CUDA tensors (one stream each) into float32
    CUDA tensors of the given (ny, nx) shapes.  With check=False returns
    (outputs, statuses) instead of raising on the first bad stream."""
    streams = [s.contiguous() for s in streams]
    dev = streams[0].device if streams else torch.device("cuda")
    outs = [torch.empty(tuple(sh), dtype=torch.float32, device=dev) for sh in shapes]
    args = DecodeArgs(streams, outs)
    rc = decompress_batch_into(args, stream)
    if check:
        _check(rc)
        return outs
    return outs, [args.status[i] for i in range(args.n)]


def decompress_batch_async(buf, offsets, lengths, shapes, stream=None, outs=None, status=None, **kw):
    """Decompress the streams buf[offsets[i] : offsets[i] + lengths[i]] (buf a
    uint8 CUDA tensor; offsets and lengths int64/uint64 CUDA tensors) into
    float32 CUDA tensors of the given shapes without waiting for the device.
    kw are the coding parameters of the streams (levels, cblk_log2w,
    cblk_log2h, spiht_tile, trunc, bypass).  Returns (outputs, status), status
    an int32 CUDA tensor of per-stream codes; both are valid once `stream`
    (default: the current stream) has reached this point.  Raises only for
    errors found before or while enqueuing."""
    n = len(shapes)
    dev = buf.device
    for t in (buf, offsets, lengths):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous()):
            raise TypeError("buf, offsets and lengths must be contiguous CUDA tensors")
    if buf.dtype != torch.uint8 or offsets.dtype not in (torch.int64, torch.uint64) or \
            lengths.dtype not in (torch.int64, torch.uint64) or offsets.numel() < n or lengths.numel() < n:
        raise TypeError("buf uint8, offsets and lengths 64-bit integers with one entry per stream")
    if outs is None:
        outs = [torch.empty(tuple(sh), dtype=torch.float32, device=dev) for sh in shapes]
    if status is None:
        status = torch.empty(max(1, n), dtype=torch.int32, device=dev)
    d_x = _arr(C.c_void_p, [o.data_ptr() for o in outs])
    ny = _arr(C.c_size_t, [int(sh[0]) for sh in shapes])
    nx = _arr(C.c_size_t, [int(sh[1]) for sh in shapes])
    p = params(**kw)
    _check(lib().ebcc_decompress_batch_async(n, C.c_void_p(buf.data_ptr()), C.c_void_p(offsets.data_ptr()),
                                             C.c_void_p(lengths.data_ptr()), d_x, ny, nx, C.byref(p),
                                             C.c_void_p(status.data_ptr()), _stream_ptr(stream)))
    return outs, status[:n]


def stream_info(header_bytes):
    """(ny, nx, mode) from the first 48 bytes of a stream (host bytes)."""
    b = (C.c_uint8 * len(header_bytes)).from_buffer_copy(bytes(header_bytes))
    ny, nx, mode = C.c_size_t(), C.c_size_t(), C.c_int()
    _check(lib().ebcc_stream_info(b, len(header_bytes), C.byref(ny), C.byref(nx), C.byref(mode)))
    return ny.value, nx.value, mode.value


def get_tuning():
    """Current kernel choices as a dict (see ebcc_tuning in include/ebcc.h)."""
    t = Tuning()
    _check(lib().ebcc_tuning_get(C.byref(t)))
    return {k: getattr(t, k) for k, _ in Tuning._fields_ if k != "struct_size"}


def set_tuning(**kw):
    """Change kernel choices (fields of ebcc_tuning: t1_encoder, t1_decoder,
    t1_wave_max, spiht, t1_lanes, t1_split, t1_persist); returns the previous
    ones."""
    old = get_tuning()
    t = Tuning()
    t.struct_size = C.sizeof(Tuning)
    for k, v in {**old, **kw}.items():
        setattr(t, k, int(v))
    _check(lib().ebcc_tuning_set(C.byref(t)))
    return old


def release():
    lib().ebcc_release()


def workspace_size(ny, nx, p=None):
    """Device bytes one compress call of an ny x nx field allocates at most
    (workspace and plan tables); 0 for invalid arguments."""
    return lib().ebcc_workspace_size(ny, nx, C.byref(p) if p is not None else None)


def workspace_size_batch(shapes, p=None, headers=None, lengths=None):
    """Workspace bytes of one batched compress (headers None) or decompress
    (headers: the 48-byte header of each stream, host bytes; lengths: the
    streams' lengths) call over fields of the given (ny, nx) shapes."""
    n = len(shapes)
    ny = _arr(C.c_size_t, [s[0] for s in shapes])
    nx = _arr(C.c_size_t, [s[1] for s in shapes])
    if headers is None:
        return lib().ebcc_workspace_size_batch(n, ny, nx, C.byref(p) if p is not None else None, None, None)
    h = b"".join(bytes(x)[:HDR_BYTES].ljust(HDR_BYTES, b"\0") for x in headers)
    hb = (C.c_uint8 * max(1, len(h))).from_buffer_copy(h or b"\0")
    ln = _arr(C.c_size_t, [int(v) for v in lengths])
    return lib().ebcc_workspace_size_batch(n, ny, nx, None, hb, ln)


def workspace_reserve(nbytes, stream=None):
    """Make the stream's library workspace exactly nbytes now."""
    _check(lib().ebcc_workspace_reserve(int(nbytes), _stream_ptr(stream)))


def device_bytes():
    """Device bytes the library holds on the current device (workspaces and
    plan tables)."""
    return lib().ebcc_device_bytes()


def profile_enable(on=True):
    lib().ebcc_profile_enable(1 if on else 0)


def profile_read():
    """{stage name: (total device ms, occurrences)} since profile_enable."""
    L = lib()
    n = L.ebcc_profile_read(None, None, 0)
    ms = (C.c_double * n)()
    calls = (C.c_long * n)()
    L.ebcc_profile_read(ms, calls, n)
    return {L.ebcc_profile_stage_name(i).decode(): (ms[i], calls[i]) for i in range(n)}
