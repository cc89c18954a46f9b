"""ctypes declarations of the C ABI in include/csv.h (argument marshalling
only; every step of the coder runs in the HIP library)."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcsv.so")

CSV_OK = 0
CSV_EINVAL = -1
CSV_EUNSUPPORTED = -2
CSV_ENOMEM = -3
CSV_EAGAIN = -4
CSV_EHIP = -5
CSV_ENOTFOUND = -6
CSV_ECANCELED = -7

CSV_FP32 = 0
CSV_BF16 = 1
CSV_FLAG_ISTA = 1
CSV_FLAG_LAMBDA_PIXEL_DOMAIN = 2
CSV_FLAG_MEASURE_INT8 = 4
CSV_FLAG_MEASURE_FP8 = 8
CSV_FLAG_TV = 16
CSV_FLAG_WHOLE_FRAME = 32
CSV_FLAG_MONOTONE = 64
CSV_FLAG_NO_QUANT = 128


class CsvParams(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("gop", C.c_int32),
                ("block", C.c_int32), ("m", C.c_int32), ("rho", C.c_float),
                ("phi_seed", C.c_uint64), ("stream_id", C.c_uint32),
                ("key_qstep", C.c_int32), ("iters", C.c_int32),
                ("lambda_frac", C.c_float), ("precision", C.c_int32),
                ("flags", C.c_int32)]


class CsvGopStream(C.Structure):
    _fields_ = [("key_levels", C.c_void_p), ("codes", C.c_void_p),
                ("exps", C.c_void_p), ("bits", C.c_void_p)]


CSV_SERVER_FAKE_EXECUTOR = 1


class CsvServerOpts(C.Structure):
    _fields_ = [("mem_budget", C.c_size_t), ("max_queue", C.c_int32),
                ("max_batch_blocks", C.c_int32), ("precision", C.c_int32),
                ("hip_streams", C.c_int32), ("flags", C.c_int32),
                ("fake_us_per_block", C.c_double), ("fake_fail_every", C.c_double)]


class CsvStats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("admitted", C.c_uint64), ("completed", C.c_uint64),
                ("rejected", C.c_uint64), ("cancelled", C.c_uint64), ("failed", C.c_uint64),
                ("recovered_pixels", C.c_uint64), ("p50_ms", C.c_double),
                ("p99_ms", C.c_double), ("mean_ms", C.c_double), ("max_ms", C.c_double),
                ("mpix_per_s", C.c_double), ("bytes_in_flight", C.c_size_t),
                ("peak_bytes", C.c_size_t), ("queue_depth", C.c_int32),
                ("batches", C.c_int32), ("max_concurrent", C.c_int32),
                ("first_arrival_s", C.c_double), ("last_done_s", C.c_double),
                ("device_bytes", C.c_size_t)]


class CsvCeilings(C.Structure):
    _fields_ = [("mfma_bf16_tflops", C.c_double), ("l2_read_tbs", C.c_double),
                ("hbm_read_tbs", C.c_double), ("lds_read_tbs", C.c_double),
                ("compute_units", C.c_int32)]


class CsvConfigPoint(C.Structure):
    _fields_ = [("gop", C.c_int32), ("m", C.c_int32), ("bits_key", C.c_uint64),
                ("bits_cs", C.c_uint64), ("cr_total", C.c_double), ("cr_key", C.c_double),
                ("cr_cs", C.c_double), ("psnr_all", C.c_double), ("psnr_cs", C.c_double),
                ("meets_floor", C.c_int32)]


class CsvError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"csv error {code}: {msg}")
        self.code = code


_P = C.POINTER
_SIGS = {
    "csv_create": (C.c_int, [_P(C.c_void_p), C.c_int, C.c_size_t]),
    "csv_destroy": (C.c_int, [C.c_void_p]),
    "csv_last_error": (C.c_char_p, []),
    "csv_version": (C.c_char_p, []),
    "csv_ctx_bytes": (C.c_int, [C.c_void_p, _P(C.c_size_t)]),
    "csv_params_default": (C.c_int, [_P(CsvParams)]),
    "csv_resolve": (C.c_int, [_P(CsvParams), _P(C.c_int32), _P(C.c_int32)]),
    "csv_encoded_size": (C.c_int, [_P(CsvParams), _P(C.c_size_t), _P(C.c_size_t),
                                   _P(C.c_size_t), _P(C.c_uint64)]),
    "csv_compression_ratio": (C.c_int, [_P(CsvParams), C.c_uint64, C.c_uint64,
                                        _P(C.c_double), _P(C.c_double), _P(C.c_double)]),
    "csv_encode_gop": (C.c_int, [C.c_void_p, _P(CsvParams), C.c_void_p,
                                 _P(CsvGopStream), C.c_void_p]),
    "csv_encode_batch": (C.c_int, [C.c_void_p, C.c_int32, _P(CsvParams), _P(C.c_void_p),
                                   _P(CsvGopStream), C.c_void_p]),
    "csv_decode_gop": (C.c_int, [C.c_void_p, _P(CsvParams), _P(CsvGopStream), C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_void_p]),
    "csv_decode_batch": (C.c_int, [C.c_void_p, C.c_int32, _P(CsvParams), _P(CsvGopStream),
                                   _P(C.c_void_p), _P(C.c_void_p), _P(C.c_void_p),
                                   C.c_void_p]),
    "csv_phi_matrix": (C.c_int, [C.c_void_p, _P(CsvParams), C.c_void_p, C.c_void_p]),
    "csv_operator_matrix": (C.c_int, [C.c_void_p, _P(CsvParams), C.c_void_p, C.c_void_p]),
    "csv_step_constant": (C.c_int, [C.c_void_p, _P(CsvParams), _P(C.c_double),
                                    _P(C.c_int32)]),
    "csv_key_encode": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_void_p]),
    "csv_key_decode": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                 C.c_void_p, C.c_void_p]),
    "csv_measure_frame": (C.c_int, [C.c_void_p, _P(CsvParams), C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "csv_measure_frame_noalloc": (C.c_int, [_P(CsvParams), C.c_void_p, C.c_void_p,
                                            C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                            C.c_void_p]),
    "csv_recover_blocks": (C.c_int, [C.c_void_p, _P(CsvParams), C.c_int32, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p]),
    "csv_profile_enable": (C.c_int, [C.c_void_p, C.c_int]),
    "csv_profile_query": (C.c_int, [C.c_void_p, C.c_char_p, _P(C.c_double), _P(C.c_int64)]),
    "csv_profile_reset": (C.c_int, [C.c_void_p]),
    "csv_probe_ceilings": (C.c_int, [C.c_void_p, _P(CsvCeilings)]),
    "csv_graph_capture": (C.c_int, [C.c_void_p, C.c_int32, _P(CsvParams), _P(CsvGopStream),
                                    _P(C.c_void_p), _P(C.c_void_p), _P(C.c_void_p), C.c_void_p,
                                    _P(C.c_void_p)]),
    "csv_graph_launch": (C.c_int, [C.c_void_p, C.c_void_p]),
    "csv_graph_destroy": (C.c_int, [C.c_void_p]),
    "csv_autotune": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                               C.c_char_p, _P(C.c_double), _P(C.c_int32), _P(C.c_int32)]),
    "csv_autotune_load": (C.c_int, [C.c_char_p]),
    "csv_autotune_choice": (C.c_int, [C.c_int32, C.c_int32, C.c_char_p, C.c_size_t,
                                      _P(C.c_int32), _P(C.c_int32)]),
    "csv_autotune_set": (C.c_int, [C.c_int32, C.c_int32, C.c_int32]),
    "csv_configure": (C.c_int, [C.c_void_p, _P(CsvParams), C.c_void_p, C.c_int32,
                                _P(C.c_int32), C.c_int32, _P(C.c_int32), C.c_int32, C.c_double,
                                _P(CsvConfigPoint), _P(C.c_int32), C.c_void_p]),
    "csv_frame_sse": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                C.c_int32, C.c_void_p, C.c_void_p]),
    "csv_clock": (C.c_double, []),
    "csv_server_create": (C.c_int, [C.c_int, _P(CsvServerOpts), _P(C.c_void_p)]),
    "csv_server_destroy": (C.c_int, [C.c_void_p]),
    "csv_server_register_stream": (C.c_int, [C.c_void_p, _P(CsvParams), _P(C.c_uint32)]),
    "csv_server_register_streams": (C.c_int, [C.c_void_p, C.c_int32, _P(CsvParams),
                                              _P(C.c_uint32)]),
    "csv_submit": (C.c_int, [C.c_void_p, C.c_uint32, _P(CsvGopStream), C.c_double,
                             _P(C.c_uint64)]),
    "csv_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.c_void_p, _P(C.c_int32)]),
    "csv_cancel": (C.c_int, [C.c_void_p, C.c_uint64]),
    "csv_server_drain": (C.c_int, [C.c_void_p, C.c_double]),
    "csv_server_stats": (C.c_int, [C.c_void_p, _P(CsvStats)]),
    "csv_server_reset_stats": (C.c_int, [C.c_void_p]),
}

_lib = None


def lib() -> C.CDLL:
    """Load libcsv.so; raises if the HIP library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"HIP library not built: {LIB_PATH} is missing "
                "(run python -m paper_1311_1419_amd.build)")
        handle = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def check(rc: int) -> None:
    if rc != CSV_OK:
        msg = lib().csv_last_error()
        raise CsvError(rc, msg.decode() if msg else "")
