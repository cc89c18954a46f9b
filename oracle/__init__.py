"""FP64 CPU oracle of the multiple-residual compressive-sensing video coder.

TEST INFRASTRUCTURE.  This package is a plain, slow, obviously correct
reference of what the HIP path computes, written from the paper (Sections 3
and 4, eqs. (1)-(4), Table I) and from the published algorithms it names or
that fill its gaps (Philox4x64-10, FISTA/MFISTA/ISTA).  Only the test suite,
the smoke check and the benchmark's CPU baseline may import it.  It shares no
code, tables or constants with the HIP library, and the library never calls
it.  Every function here is pinned by a test against something other than
itself (numpy's own Philox, scipy's DCT, eigvalsh, KKT conditions, brute
force, scikit-learn's Lasso, Table I).
"""
from . import codec, cs, keyframe, philox
from .codec import Params, GopStream, Decoded, encode_gop, decode_gop, psnr

__all__ = ["codec", "cs", "keyframe", "philox", "Params", "GopStream",
           "Decoded", "encode_gop", "decode_gop", "psnr"]
