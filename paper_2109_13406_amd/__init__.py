"""mpdd: double-double Rgemm / Rsyrk on AMD Instinct MI355X (gfx950).

The compute path is libmpdd.so (hand-written HIP kernels behind the C ABI in
include/mpdd.h); `binding` marshals arguments to it with ctypes (torch
supplies device memory and streams only); `loadgen` drives the request
server and `autotune` writes tile tables for it.  Importing this package
does not load the library; the first call does, and raises if it is
missing.
"""
from .binding import (MPDD_OZAKI_CRT, MPDD_OZAKI_F64, MPDD_OZAKI_I8, MPDD_PLAIN,  # noqa
                      MPDD_PLAIN_ACCURATE,
                      load, mpdd_create, mpdd_destroy, mpdd_Rgemm, mpdd_Rgemm_ex,
                      mpdd_Rgemm_host, mpdd_Rgemm_host_ex, mpdd_Rgemm_noalloc, mpdd_Rsyrk,
                      mpdd_Rsyrk_ex, mpdd_Rsyrk_host, mpdd_Rsyrk_host_ex, mpdd_Cgemm, mpdd_Qgemm, mpdd_Rpotrf,
                      mpdd_ozaki_crt_exponent, mpdd_ozaki_digit_widths,
                      mpdd_ozaki_split, mpdd_tile_count, mpdd_tile_info, mpdd_version)
