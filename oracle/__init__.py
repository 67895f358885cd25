"""Plain, slow FP64 CPU oracle for multiplication-avoiding power iteration (MAPI).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or link
this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (``paper_2110_12065_amd``) and imports nothing from it.

Every function follows a passage of Pan, Badawi, Miao, Koyuncu, Cetin,
"Multiplication-Avoiding Variant of Power Iteration with Applications"
(arXiv 2110.12065), cited by section / equation / algorithm.  Arithmetic is
IEEE float64 (numpy) with loops in index order; a library primitive (numpy
sum, matmul) serves as a step where the definition is a plain sum or product.

Pinned by the ``-m "not gpu"`` tests in ``tests/test_oracle_*.py``; see the
header of each module for what pins which function and for the functions
whose parity is unpinned.
"""
from .core import (  # noqa: F401
    OracleDegenerate,
    term_min1, term_min2, term_diamond, term_dot, TERMS,
    vec_product, mavp, mapi, rpi, hybrid, normalize_l2, ranks,
)
from .pca import covariance, mingram, mingram_entry, deflate_projection, pca_topk  # noqa: F401
from .pagerank import (  # noqa: F401
    dangling_mask, dense_G, pagerank_mavp_dense, pagerank_mavp_csr,
    pagerank_rpi_csr, pagerank,
)
from .minibatch import minibatch_mapi  # noqa: F401
from .factored import factored_product, factored_mapi  # noqa: F401
from .image import min_outer, minouter_deflate, minouter_reconstruct, image_reconstruct, psnr  # noqa: F401
from .quant import (  # noqa: F401
    bf16_decode, bf16_encode, e4m3fn_table, e4m3fn_decode, e4m3fn_encode,
    fp8_row_scale, fp8_rows_quantize, fp8_rows_dequantize, bf16_quantize, bf16_dequantize,
    E4M3_MAX,
)
