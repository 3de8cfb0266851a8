"""MI355X chunk video codec (DCVC-UF hot path) - Python binding of libufvc.

Argument marshalling only: every step of encode / decode runs in the HIP
kernels of ``libufvc.so``.  PyTorch provides device memory and streams; tensors
are passed to the C ABI as raw device pointers.  Importing this package loads
the library and raises if it is missing (build it with
``python paper_2606_04410_amd/build.py``).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

try:
    # PyTorch carries its own HIP runtime; loaded first, it is the one the
    # library binds to as well, so torch's device memory and streams and the
    # library's calls share one runtime whichever module the caller imports
    # first.
    import torch  # noqa: F401
except ImportError:  # the library alone (host-side calls, symbol checks)
    pass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libufvc.so")

FP32, BF16, BF16_FP8 = 0, 1, 2
PRECISIONS = {"fp32": FP32, "bf16": BF16, "bf16_fp8": BF16_FP8}
STATUS = {0: "OK", -1: "INVAL", -2: "NOSPC", -3: "CORRUPT", -4: "DEVICE", -5: "NOMEM",
          -6: "UNSUPPORTED", -7: "SCRATCH"}
BUF_Y, BUF_ZSYM, BUF_PARAMS, BUF_IDX, BUF_SYM, BUF_D2, BUF_F, BUF_K1, BUF_K2, BUF_AMAX = range(10)
Z_CHANNELS = 32
# Segment sizes (log2 symbols per rANS segment) used unless a codec names its
# own: the 1080p benchmark configuration.  Each segment carries 32 final lane
# states (128 bytes) and is one chain of 2^seg_log2 / 32 serial decode steps,
# so smaller segments buy decoder parallelism for stream size.  Measured at
# 1080p T=8 (bench.py --seg-sweep): 2^12 decodes y in 67 us against 120 us
# at 2^13 for 1.6% more bytes; 2^11 is no faster (two decoder blocks per CU
# already run every segment pair of 2^12 at once) and costs 4.8%.
DEFAULT_SEG_LOG2 = 12
DEFAULT_SEG_LOG2_Z = 10


class UfvcError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {STATUS.get(code, code)}")
        self.code = code


class _Config(ctypes.Structure):
    _fields_ = [("T", ctypes.c_int), ("C", ctypes.c_int), ("precision", ctypes.c_int),
                ("seg_log2", ctypes.c_int), ("seg_log2_z", ctypes.c_int),
                ("model_tag", ctypes.c_uint32), ("autotune", ctypes.c_int),
                ("quadtree", ctypes.c_int), ("temporal", ctypes.c_int)]


class _Chunk(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int), ("H", ctypes.c_int), ("W", ctypes.c_int),
                ("frames", ctypes.c_void_p), ("frames_out", ctypes.c_void_p),
                ("bitstream", ctypes.c_void_p), ("capacity", ctypes.c_size_t),
                ("len", ctypes.c_size_t), ("status", ctypes.c_int)]


class _ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("lanes", ctypes.c_int),
                ("max_batch", ctypes.c_int), ("use_graph", ctypes.c_int),
                ("small_pixels", ctypes.c_int)]


class _Request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("model", ctypes.c_int), ("H", ctypes.c_int),
                ("W", ctypes.c_int), ("frames", ctypes.c_void_p), ("frames_out", ctypes.c_void_p),
                ("bitstream", ctypes.c_void_p), ("capacity", ctypes.c_size_t),
                ("len", ctypes.c_size_t), ("tag", ctypes.c_uint64)]


class _Completion(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("tag", ctypes.c_uint64), ("status", ctypes.c_int),
                ("batch_size", ctypes.c_int), ("len", ctypes.c_size_t),
                ("t_submit_us", ctypes.c_double), ("t_admit_us", ctypes.c_double),
                ("t_done_us", ctypes.c_double)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing; build it with python paper_2606_04410_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    P, S, I, U = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_uint32
    sigs = {
        "ufvc_weight_count": (S, [I, I]),
        "ufvc_create": (I, [ctypes.POINTER(_Config), P, S, ctypes.POINTER(P)]),
        "ufvc_destroy": (None, [P]),
        "ufvc_max_bitstream_bytes": (S, [P, I, I]),
        "ufvc_encode_chunk": (I, [P, P, I, I, I, P, S, ctypes.POINTER(S), P]),
        "ufvc_decode_chunk": (I, [P, P, S, I, I, I, P, P]),
        "ufvc_sync_status": (I, [P, P]),
        "ufvc_stream_create": (I, [P, I, I, ctypes.POINTER(P)]),
        "ufvc_stream_destroy": (None, [P]),
        "ufvc_stream_reset": (I, [P]),
        "ufvc_stream_copy_context": (I, [P, P, S]),
        "ufvc_encode_next": (I, [P, P, P, S, ctypes.POINTER(S), P]),
        "ufvc_decode_next": (I, [P, P, S, P, P]),
        "ufvc_get_tables": (I, [P, P, P, P]),
        "ufvc_rans_encode": (I, [P, P, P, S, I, P, S, ctypes.POINTER(S), P]),
        "ufvc_rans_encode_noalloc": (I, [P, P, P, S, I, P, S, ctypes.POINTER(S), P]),
        "ufvc_rans_decode": (I, [P, P, S, P, S, I, P, P]),
        "ufvc_synthesize": (I, [P, P, I, I, I, P, P]),
        "ufvc_convert_frames": (I, [P, I, P, I, I, I, I, P]),
        "ufvc_copy_buffer": (I, [P, I, P, S]),
        "ufvc_profile_enable": (I, [P, I]),
        "ufvc_profile_stage_count": (I, []),
        "ufvc_profile_stage_name": (ctypes.c_char_p, [I]),
        "ufvc_profile_read": (I, [P, P, P, I]),
        "ufvc_get_tuning": (I, [P, I, I, P, I]),
        "ufvc_tile_config": (I, [I, P, P, P]),
        "ufvc_num_tile_configs": (I, []),
        "ufvc_force_tile_config": (I, [P, I]),
        "ufvc_dcblock_create": (I, [I, P, S, ctypes.POINTER(P)]),
        "ufvc_dcblock_destroy": (None, [P]),
        "ufvc_dcblock_run": (I, [P, P, P, I, I, P]),
        "ufvc_batch_create": (I, [P, I, ctypes.POINTER(P)]),
        "ufvc_batch_destroy": (None, [P]),
        "ufvc_encode_batch": (I, [P, P, I, P]),
        "ufvc_decode_batch": (I, [P, P, I, I, P]),
        "ufvc_batch_sync_status": (I, [P, P, I, P]),
        "ufvc_batch_set_policy": (I, [P, I]),
        "ufvc_batch_stats": (I, [P, P, I]),
        "ufvc_server_create": (I, [P, I, ctypes.POINTER(_ServerConfig), ctypes.POINTER(P)]),
        "ufvc_server_submit": (I, [P, ctypes.POINTER(_Request), ctypes.POINTER(ctypes.c_uint64)]),
        "ufvc_server_poll": (I, [P, P, I, I]),
        "ufvc_server_stats": (I, [P, P, I]),
        "ufvc_server_destroy": (None, [P]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    del U
    return lib


lib = _load()

# Names of the exported entry points (what include/ufvc.h declares).
EXPORTS = ("ufvc_weight_count", "ufvc_create", "ufvc_destroy", "ufvc_max_bitstream_bytes",
           "ufvc_encode_chunk", "ufvc_decode_chunk", "ufvc_sync_status", "ufvc_stream_create",
           "ufvc_stream_destroy", "ufvc_stream_reset", "ufvc_stream_copy_context",
           "ufvc_encode_next", "ufvc_decode_next", "ufvc_get_tables",
           "ufvc_rans_encode", "ufvc_rans_encode_noalloc", "ufvc_rans_decode", "ufvc_synthesize", "ufvc_copy_buffer",
           "ufvc_profile_enable", "ufvc_profile_stage_count", "ufvc_profile_stage_name",
           "ufvc_profile_read", "ufvc_get_tuning", "ufvc_tile_config", "ufvc_num_tile_configs",
           "ufvc_force_tile_config", "ufvc_convert_frames", "ufvc_dcblock_create",
           "ufvc_dcblock_destroy", "ufvc_dcblock_run", "ufvc_batch_create",
           "ufvc_batch_destroy", "ufvc_encode_batch", "ufvc_decode_batch", "ufvc_batch_sync_status",
           "ufvc_batch_set_policy", "ufvc_batch_stats",
           "ufvc_server_create", "ufvc_server_submit", "ufvc_server_poll", "ufvc_server_stats",
           "ufvc_server_destroy")
REQ_ENCODE, REQ_DECODE = 0, 1
FMT_YUV444, FMT_RGB709, FMT_YUV420 = 0, 1, 2
FORMATS = {"yuv444": FMT_YUV444, "rgb": FMT_RGB709, "yuv420": FMT_YUV420}


def frame_elems(fmt: str, T: int, H: int, W: int) -> int:
    """float32 values of T frames of H x W in a format."""
    return T * H * W * 3 if fmt != "yuv420" else T * H * W * 3 // 2


def convert_frames(src, src_fmt: str, dst_fmt: str, T: int, H: int, W: int, out=None,
                   stream=None):
    """Format conversion on the GPU (ufvc_convert_frames); src and the result
    are cuda float32 (T, 3, H, W) for yuv444 / rgb, flat (T * 1.5 H W) for
    yuv420."""
    import torch
    if out is None:
        shape = (T, 3, H, W) if dst_fmt != "yuv420" else (frame_elems("yuv420", T, H, W),)
        out = torch.empty(shape, dtype=torch.float32, device=src.device)
    assert src.is_contiguous() and out.is_contiguous()
    assert src.numel() == frame_elems(src_fmt, T, H, W) and out.numel() == frame_elems(dst_fmt, T, H, W)
    _check(lib.ufvc_convert_frames(_ptr(src), FORMATS[src_fmt], _ptr(out), FORMATS[dst_fmt], T, H, W,
                                   _stream(stream)), "ufvc_convert_frames")
    return out
TUNED_LAYERS = ("a1", "a2", "a3", "d1", "d2", "d3", "k1", "k2", "k3")


def layer_order(T: int, quadtree: bool = False, temporal: bool = False) -> list[str]:
    """Layer names in the order ufvc_create expects them."""
    names = ["a1", "a2", "a3", "h", "p", "d1", "d2", "d3"]
    for t in range(T):
        names += [f"k1_{t}", f"k2_{t}", f"k3_{t}"]
    if quadtree:
        names += ["m1", "m2", "m3"]
    if temporal:
        names += ["c1", "c2", "a1c", "pc", "d1c"]
    return names


def flatten_weights(weights: dict, T: int, quadtree: bool = False,
                    temporal: bool = False) -> np.ndarray:
    return np.ascontiguousarray(
        np.concatenate([np.asarray(weights[n], np.float32).reshape(-1)
                        for n in layer_order(T, quadtree, temporal)]))


def _check(code: int, what: str):
    if code != 0:
        raise UfvcError(code, what)


def _ptr(t) -> int:
    return t.data_ptr()


def _stream(stream) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class Codec:
    """One codec context (one model: fixed T and C) on the current device."""

    def __init__(self, T: int, C: int, weights: dict, precision: str = "bf16",
                 seg_log2: int = None, seg_log2_z: int = None, model_tag: int = 0,
                 autotune: bool = False, quadtree: bool = None, temporal: bool = None):
        """quadtree: four-step progressive means over the quadtree partition;
        temporal: chunks coded with their stream's temporal context (through
        Stream objects).  Each is on by default exactly when the weights hold
        its layers (m1..m3; c1, c2, a1c, pc, d1c)."""
        self.T, self.C = T, C
        self.quadtree = ("m1" in weights) if quadtree is None else bool(quadtree)
        self.temporal = ("c1" in weights) if temporal is None else bool(temporal)
        self.precision = precision
        seg_log2 = DEFAULT_SEG_LOG2 if seg_log2 is None else seg_log2
        seg_log2_z = DEFAULT_SEG_LOG2_Z if seg_log2_z is None else seg_log2_z
        self.seg_log2, self.seg_log2_z, self.model_tag = seg_log2, seg_log2_z, model_tag
        flat = flatten_weights(weights, T, self.quadtree, self.temporal)
        cfg = _Config(T, C, PRECISIONS[precision], seg_log2, seg_log2_z, model_tag & 0xFFFFFFFF,
                      1 if autotune else 0, 1 if self.quadtree else 0, 1 if self.temporal else 0)
        h = ctypes.c_void_p()
        _check(lib.ufvc_create(ctypes.byref(cfg), flat.ctypes.data, flat.size, ctypes.byref(h)),
               "ufvc_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib.ufvc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- sizes
    def latent_size(self, H: int, W: int):
        Hp, Wp = -(-H // 16) * 16, -(-W // 16) * 16
        h, w = Hp // 8, Wp // 8
        return h, w, -(-h // 2), -(-w // 2)

    def max_bitstream_bytes(self, H: int, W: int) -> int:
        return int(lib.ufvc_max_bitstream_bytes(self._h, H, W))

    # ----------------------------------------------------------- coding API
    def encode(self, frames, out=None, stream=None, fmt: str = "yuv444", H: int = None,
               W: int = None):
        """frames: cuda float32 (T, 3, H, W) YUV444 planes (the codec's
        interface); fmt "rgb" (BT.709) or "yuv420" (flat, give H and W)
        converts on the GPU first.  Returns (uint8 cuda buffer, nbytes)."""
        import torch
        if fmt != "yuv444":
            if fmt == "rgb":
                H, W = frames.shape[2], frames.shape[3]
            frames = convert_frames(frames, fmt, "yuv444", self.T, H, W, stream=stream)
        T, _, H, W = frames.shape
        assert frames.is_cuda and frames.dtype == torch.float32 and frames.is_contiguous()
        if out is None:
            out = torch.empty(self.max_bitstream_bytes(H, W), dtype=torch.uint8, device=frames.device)
        n = ctypes.c_size_t(0)
        code = lib.ufvc_encode_chunk(self._h, _ptr(frames), T, H, W, _ptr(out), out.numel(),
                                     ctypes.byref(n), _stream(stream))
        _check(code, "ufvc_encode_chunk")
        return out, n.value

    def decode(self, bitstream, nbytes: int, H: int, W: int, out=None, stream=None, check=True,
               fmt: str = "yuv444"):
        """bitstream: cuda uint8.  Returns cuda float32 (T, 3, H, W) YUV444
        planes, or the frames converted on the GPU to fmt ("rgb", or "yuv420"
        as a flat array)."""
        import torch
        yuv = out if (out is not None and fmt == "yuv444") else None
        if yuv is None:
            yuv = torch.empty((self.T, 3, H, W), dtype=torch.float32, device=bitstream.device)
        _check(lib.ufvc_decode_chunk(self._h, _ptr(bitstream), nbytes, self.T, H, W, _ptr(yuv),
                                     _stream(stream)), "ufvc_decode_chunk")
        res = yuv
        if fmt != "yuv444":
            res = convert_frames(yuv, "yuv444", fmt, self.T, H, W, out=out, stream=stream)
        if check:
            self.sync_status(stream)
        return res

    def sync_status(self, stream=None):
        _check(lib.ufvc_sync_status(self._h, _stream(stream)), "decode status")

    def status(self, stream=None) -> int:
        return int(lib.ufvc_sync_status(self._h, _stream(stream)))

    def synthesize(self, y_hat_hwc, H: int, W: int, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty((self.T, 3, H, W), dtype=torch.float32, device=y_hat_hwc.device)
        _check(lib.ufvc_synthesize(self._h, _ptr(y_hat_hwc), self.T, H, W, _ptr(out),
                                   _stream(stream)), "ufvc_synthesize")
        return out

    # ------------------------------------------------------- stage access
    def tables(self):
        freq = np.zeros((64, 65), np.uint16)
        cum = np.zeros((64, 65), np.uint16)
        thr = np.zeros(63, np.float32)
        _check(lib.ufvc_get_tables(self._h, freq.ctypes.data, cum.ctypes.data, thr.ctypes.data),
               "ufvc_get_tables")
        return freq, cum, thr

    def rans_encode(self, sym, idx, seg_log2: int, stream=None):
        """sym, idx: cuda uint8 (n,).  Returns bytes: u32 seg_bytes[n_seg] + segments."""
        import torch
        n = sym.numel()
        nseg = -(-n // (1 << seg_log2))
        cap = 4 * nseg + nseg * 132 + 2 * n + 16
        out = torch.empty(cap, dtype=torch.uint8, device=sym.device)
        ln = ctypes.c_size_t(0)
        _check(lib.ufvc_rans_encode(self._h, _ptr(sym), _ptr(idx), n, seg_log2, _ptr(out), cap,
                                    ctypes.byref(ln), _stream(stream)), "ufvc_rans_encode")
        return out[:ln.value]

    def rans_encode_noalloc(self, sym, idx, seg_log2: int, out=None, stream=None):
        """As rans_encode through the allocation-free entry point (its scratch
        is the library's fixed per-GPU array).  Returns a view of `out`."""
        import torch
        n = sym.numel()
        nseg = -(-n // (1 << seg_log2))
        cap = 4 * nseg + nseg * 132 + 2 * n + 16
        if out is None:
            out = torch.empty(cap, dtype=torch.uint8, device=sym.device)
        ln = ctypes.c_size_t(0)
        _check(lib.ufvc_rans_encode_noalloc(self._h, _ptr(sym), _ptr(idx), n, seg_log2, _ptr(out),
                                            out.numel(), ctypes.byref(ln), _stream(stream)),
               "ufvc_rans_encode_noalloc")
        return out[:ln.value]

    def rans_decode(self, data, idx, seg_log2: int, stream=None):
        import torch
        n = idx.numel()
        sym = torch.empty(n, dtype=torch.uint8, device=idx.device)
        _check(lib.ufvc_rans_decode(self._h, _ptr(data), data.numel(), _ptr(idx), n, seg_log2,
                                    _ptr(sym), _stream(stream)), "ufvc_rans_decode")
        return sym

    def tuning(self, H: int, W: int) -> dict:
        """{layer: (config index, tile rows, tile cols, channels)} chosen so far."""
        cfg = np.zeros(9, np.int32)
        _check(lib.ufvc_get_tuning(self._h, H, W, cfg.ctypes.data, 9), "ufvc_get_tuning")
        out = {}
        for name, k in zip(TUNED_LAYERS, cfg):
            if k < 0:
                out[name] = None
                continue
            th, tw, bn = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
            lib.ufvc_tile_config(int(k), ctypes.byref(th), ctypes.byref(tw), ctypes.byref(bn))
            out[name] = (int(k), th.value, tw.value, bn.value)
        return out

    def force_tile_config(self, cfg: int):
        """Test hook: every conv layer that supports tile configuration cfg uses
        it (-1 restores the tuned / default choice)."""
        _check(lib.ufvc_force_tile_config(self._h, int(cfg)), "ufvc_force_tile_config")

    # ------------------------------------------------------------ timing
    def profile(self, on: bool = True):
        _check(lib.ufvc_profile_enable(self._h, 1 if on else 0), "ufvc_profile_enable")

    def profile_read(self) -> dict:
        """{stage name: (total ms, launches)} since the last read / enable."""
        n = lib.ufvc_profile_stage_count()
        tot = np.zeros(n, np.float64)
        cnt = np.zeros(n, np.int32)
        _check(lib.ufvc_profile_read(self._h, tot.ctypes.data, cnt.ctypes.data, n), "ufvc_profile_read")
        return {lib.ufvc_profile_stage_name(i).decode(): (float(tot[i]), int(cnt[i]))
                for i in range(n) if cnt[i]}

    def buffer(self, which: int, H: int, W: int) -> np.ndarray:
        h, w, hz, wz = self.latent_size(H, W)
        C = self.C
        act = np.float32 if self.precision == "fp32" else np.uint16
        shape, dt = {BUF_Y: ((h, w, C), np.float32), BUF_ZSYM: ((hz, wz, Z_CHANNELS), np.uint8),
                     BUF_PARAMS: ((h, w, 2 * C), np.float32), BUF_IDX: ((h, w, C), np.uint8),
                     BUF_SYM: ((h, w, C), np.uint8), BUF_D2: ((h, w, C), act),
                     BUF_F: ((h, w, C), act), BUF_K1: ((h, w, self.T * C), act),
                     BUF_K2: ((h, w, self.T * C), act), BUF_AMAX: ((8,), np.uint32)}[which]
        a = np.zeros(shape, dt)
        _check(lib.ufvc_copy_buffer(self._h, which, a.ctypes.data, a.nbytes), "ufvc_copy_buffer")
        if a.dtype == np.uint16:      # bfloat16 bits -> float32
            a = (a.astype(np.uint32) << 16).view(np.float32)
        elif which == BUF_AMAX:
            a = a.view(np.float32)
        return a


class Stream:
    """The temporal context of one video stream at one size, on one side
    (encoder or decoder) of a temporal model: chunks go through it in stream
    order.  Keep the codec alive while the stream is."""

    def __init__(self, codec: "Codec", H: int, W: int):
        self.codec, self.H, self.W = codec, H, W
        h = ctypes.c_void_p()
        _check(lib.ufvc_stream_create(codec._h, H, W, ctypes.byref(h)), "ufvc_stream_create")
        self._h = h

    def encode(self, frames, out=None, stream=None):
        """Next chunk: cuda float32 (T, 3, H, W).  Returns (uint8 buffer, nbytes)."""
        import torch
        assert frames.is_cuda and frames.dtype == torch.float32 and frames.is_contiguous()
        if out is None:
            out = torch.empty(self.codec.max_bitstream_bytes(self.H, self.W), dtype=torch.uint8,
                              device=frames.device)
        n = ctypes.c_size_t(0)
        _check(lib.ufvc_encode_next(self._h, _ptr(frames), _ptr(out), out.numel(), ctypes.byref(n),
                                    _stream(stream)), "ufvc_encode_next")
        return out, n.value

    def decode(self, bitstream, nbytes: int, out=None, stream=None, check=True):
        import torch
        if out is None:
            out = torch.empty((self.codec.T, 3, self.H, self.W), dtype=torch.float32,
                              device=bitstream.device)
        _check(lib.ufvc_decode_next(self._h, _ptr(bitstream), nbytes, _ptr(out), _stream(stream)),
               "ufvc_decode_next")
        if check:
            self.codec.sync_status(stream)
        return out

    def context(self) -> np.ndarray:
        """The next chunk's context, (h, w, C) float32."""
        h, w, _, _ = self.codec.latent_size(self.H, self.W)
        C = self.codec.C
        act = np.float32 if self.codec.precision == "fp32" else np.uint16
        a = np.zeros((h, w, C), act)
        _check(lib.ufvc_stream_copy_context(self._h, a.ctypes.data, a.nbytes), "ufvc_stream_copy_context")
        if a.dtype == np.uint16:
            a = (a.astype(np.uint32) << 16).view(np.float32)
        return a

    def reset(self):
        _check(lib.ufvc_stream_reset(self._h), "ufvc_stream_reset")

    def close(self):
        if getattr(self, "_h", None):
            lib.ufvc_stream_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


DC_BLOCK_LAYERS = ("pw1", "dw", "pw2", "pw3", "pw4")


class DcBlock:
    """One fused DC block (depth-wise 3x3 between point-wise mixings, then a
    point-wise feed-forward stage) on bf16 [h][w][C] feature maps."""

    def __init__(self, C: int, weights: dict):
        self.C = C
        flat = np.ascontiguousarray(np.concatenate(
            [np.asarray(weights[n], np.float32).reshape(-1) for n in DC_BLOCK_LAYERS]))
        h = ctypes.c_void_p()
        _check(lib.ufvc_dcblock_create(C, flat.ctypes.data, flat.size, ctypes.byref(h)),
               "ufvc_dcblock_create")
        self._h = h

    def run(self, x, out=None, stream=None):
        """x: cuda bfloat16 (h, w, C) contiguous.  Returns bfloat16 (h, w, C)."""
        import torch
        assert x.is_cuda and x.dtype == torch.bfloat16 and x.is_contiguous() and x.shape[2] == self.C
        if out is None:
            out = torch.empty_like(x)
        _check(lib.ufvc_dcblock_run(self._h, _ptr(x), _ptr(out), x.shape[0], x.shape[1],
                                    _stream(stream)), "ufvc_dcblock_run")
        return out

    def close(self):
        if getattr(self, "_h", None):
            lib.ufvc_dcblock_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many chunks per launch over one or more models (contexts) sharing C,
    precision and segment sizes.  Keep the codecs alive while the batch is."""

    def __init__(self, codecs):
        self.codecs = list(codecs)
        arr = (ctypes.c_void_p * len(self.codecs))(*[c._h.value for c in self.codecs])
        h = ctypes.c_void_p()
        _check(lib.ufvc_batch_create(arr, len(self.codecs), ctypes.byref(h)), "ufvc_batch_create")
        self._h = h
        self._last = None

    def close(self):
        if getattr(self, "_h", None):
            lib.ufvc_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def encode(self, items, stream=None):
        """items: [(model index, frames cuda (T,3,H,W), out uint8 cuda buffer)].
        Returns the coded lengths."""
        n = len(items)
        arr = (_Chunk * n)()
        for i, (m, fr, out) in enumerate(items):
            arr[i] = _Chunk(m, fr.shape[2], fr.shape[3], _ptr(fr), None, _ptr(out), out.numel(), 0, 0)
        code = lib.ufvc_encode_batch(self._h, arr, n, _stream(stream))
        _check(code, "ufvc_encode_batch")
        return [int(arr[i].len) for i in range(n)]

    def decode(self, items, graph=False, stream=None, check=True):
        """items: [(model index, bitstream cuda, nbytes, H, W, frames_out cuda)]."""
        n = len(items)
        arr = (_Chunk * n)()
        for i, (m, bs, nb, H, W, out) in enumerate(items):
            arr[i] = _Chunk(m, H, W, None, _ptr(out), _ptr(bs), 0, nb, 0)
        self._last = arr
        _check(lib.ufvc_decode_batch(self._h, arr, n, 1 if graph else 0, _stream(stream)),
               "ufvc_decode_batch")
        if check:
            return self.sync_status(stream)
        return None

    def set_policy(self, policy: int):
        """0: one launch per tile configuration in a stage; 1: one launch per
        stage (drops cached plans)."""
        _check(lib.ufvc_batch_set_policy(self._h, int(policy)), "ufvc_batch_set_policy")

    def stats(self):
        v = (ctypes.c_uint64 * 6)()
        _check(lib.ufvc_batch_stats(self._h, v, 6), "ufvc_batch_stats")
        return dict(plans_built=v[0], plans_evicted=v[1], plans_cached=v[2], conv_stages=v[3],
                    conv_launches=v[4], policy=v[5])

    def sync_status(self, stream=None):
        arr = self._last
        code = lib.ufvc_batch_sync_status(self._h, arr, len(arr), _stream(stream))
        return [int(arr[i].status) for i in range(len(arr))], code


class Server:
    """Continuous-batching request server over one or more codecs (sharing C,
    precision and segment sizes).  Requests carry device tensors that the
    caller keeps alive until their completion is polled."""

    def __init__(self, codecs, hbm_budget: int = 0, lanes: int = 2, max_batch: int = 8,
                 graph: bool = True, small_pixels: int = 0):
        self.codecs = list(codecs)
        arr = (ctypes.c_void_p * len(self.codecs))(*[c._h.value for c in self.codecs])
        cfg = _ServerConfig(hbm_budget, lanes, max_batch, 1 if graph else 0, small_pixels)
        h = ctypes.c_void_p()
        _check(lib.ufvc_server_create(arr, len(self.codecs), ctypes.byref(cfg), ctypes.byref(h)),
               "ufvc_server_create")
        self._h = h
        self._keep = {}

    def submit_encode(self, model: int, frames, out, tag: int = 0) -> int:
        r = _Request(REQ_ENCODE, model, frames.shape[2], frames.shape[3], _ptr(frames), None,
                     _ptr(out), out.numel(), 0, tag)
        return self._submit(r, (frames, out))

    def submit_decode(self, model: int, bitstream, nbytes: int, H: int, W: int, out,
                      tag: int = 0) -> int:
        r = _Request(REQ_DECODE, model, H, W, None, _ptr(out), _ptr(bitstream), 0, nbytes, tag)
        return self._submit(r, (bitstream, out))

    def _submit(self, r, keep) -> int:
        t = ctypes.c_uint64()
        _check(lib.ufvc_server_submit(self._h, ctypes.byref(r), ctypes.byref(t)), "ufvc_server_submit")
        self._keep[t.value] = keep
        return t.value

    def poll(self, max_n: int = 64, timeout_ms: int = 100):
        """Completions as dicts (ticket, tag, status, batch_size, len, times in us)."""
        arr = (_Completion * max_n)()
        k = lib.ufvc_server_poll(self._h, arr, max_n, timeout_ms)
        if k < 0:
            _check(k, "ufvc_server_poll")
        out = []
        for i in range(k):
            c = arr[i]
            self._keep.pop(c.ticket, None)
            out.append(dict(ticket=c.ticket, tag=c.tag, status=c.status, batch_size=c.batch_size,
                            len=c.len, t_submit_us=c.t_submit_us, t_admit_us=c.t_admit_us,
                            t_done_us=c.t_done_us))
        return out

    def stats(self):
        v = (ctypes.c_uint64 * 8)()
        _check(lib.ufvc_server_stats(self._h, v, 8), "ufvc_server_stats")
        return dict(queued=v[0], in_flight=v[1], completed=v[2], batches=v[3],
                    peak_footprint=v[4], budget=v[5], plans_built=v[6], arena_bytes=v[7])

    def close(self):
        if getattr(self, "_h", None):
            lib.ufvc_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
