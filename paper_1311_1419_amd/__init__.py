"""MI355X (gfx950) multiple-residual compressive-sensing video coder.

The coder of Yu, Qiao, Luo and Yang (key frame + CS frames per GOP,
closed-loop residual against the decoded key frame, random measurement,
sparse recovery, eq. (4) reconstruction), with the encode/decode hot path in
hand-written HIP behind a C ABI (include/csv.h).  This package only
marshals arguments: it loads libcsv.so and fails loudly if it is missing.
"""
from ._native import (CSV_BF16, CSV_FP32, CSV_FLAG_ISTA, CSV_FLAG_LAMBDA_PIXEL_DOMAIN,
                      CSV_FLAG_MEASURE_FP8, CSV_FLAG_MEASURE_INT8, CSV_FLAG_TV,
                      CSV_FLAG_WHOLE_FRAME, CSV_FLAG_MONOTONE, CSV_FLAG_NO_QUANT, CsvError,
                      lib)
from .api import (Context, GopStream, Params, kernel_choice, load_kernel_choices,
                  measure_frame_noalloc, set_kernel_choice)
from .server import Server, clock

__all__ = ["Context", "GopStream", "Params", "Server", "clock", "kernel_choice",
           "measure_frame_noalloc",
           "load_kernel_choices", "set_kernel_choice", "CsvError", "CSV_BF16", "CSV_FP32",
           "CSV_FLAG_ISTA", "CSV_FLAG_LAMBDA_PIXEL_DOMAIN", "CSV_FLAG_MEASURE_INT8",
           "CSV_FLAG_MEASURE_FP8", "CSV_FLAG_TV",
           "CSV_FLAG_WHOLE_FRAME", "CSV_FLAG_MONOTONE", "CSV_FLAG_NO_QUANT", "lib"]
