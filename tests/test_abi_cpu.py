"""The C ABI library loads and exports every function include/glasso.h declares;
struct layouts of the Python binding match the C compiler's (CPU only)."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "glasso.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(glasso_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_2205_10027_amd import _native

    lib = ctypes.CDLL(_native.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 11
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding declares a signature for each of them
    assert set(names) <= set(_native.SIGNATURES)


def test_host_only_entry_points():
    import paper_2205_10027_amd as g

    lib = g._lib
    assert lib.glasso_error_string(0) == b"success"
    assert lib.glasso_error_string(2) == b"matrix is not positive definite"
    opt = g.GlassoOptions()
    assert lib.glasso_default_options(ctypes.byref(opt)) == 0
    assert (opt.max_iter, opt.t0, opt.shrink, opt.t_floor) == (500, 1.0, 0.5, 1e-4)
    # workspace: 9 padded FP64 matrices + int8 mask + small vectors
    b = g.workspace_bytes(10000)
    np_ = 10112
    assert 9 * np_ * np_ * 8 < b < 9 * np_ * np_ * 8 + 2 * np_ * np_ + 64 * 2**20
    with pytest.raises(g.GlassoError):
        g.workspace_bytes(0)
    # up to n = 2048 the line search holds 4 trial points and factors per problem
    b1, np1 = g.workspace_bytes(1000), 1024
    assert 15 * np1 * np1 * 8 < b1 < 15 * np1 * np1 * 8 + 2 * np1 * np1 + 64 * 2**20
    assert opt.ls_width == 0
    # the mixed forms keep their reduced-precision operands inside the FP64 buffers
    assert g.workspace_bytes(10000, "fp32") == g.workspace_bytes(10000, "bf16x3") == b
    with pytest.raises(g.GlassoError):
        g.workspace_bytes(100, 3)
    assert lib.glasso_create(None, None) == 1
    # the allocation-free small solve checks its arguments on the host first
    assert lib.glasso_solve_small_static(None, 0, None, None, None, 1e-6, None, None, None, None) == 1
    assert g.SMALL_STATIC_MAX_COUNT == 16384
    # option checks run before any device call
    assert opt.tile_policy == g.TILES_AUTO == -1 and opt.graphs == 0 and opt.w_mixed == -1
    h = ctypes.c_void_p()
    bad = g.GlassoOptions()
    lib.glasso_default_options(ctypes.byref(bad))
    bad.tile_policy = -2
    assert lib.glasso_create(ctypes.byref(h), ctypes.byref(bad)) == 1 and not h.value
    lib.glasso_default_options(ctypes.byref(bad))
    bad.precision = 3
    assert lib.glasso_create(ctypes.byref(h), ctypes.byref(bad)) == 1 and not h.value
    for width in (-1, 17):
        lib.glasso_default_options(ctypes.byref(bad))
        bad.ls_width = width
        assert lib.glasso_create(ctypes.byref(h), ctypes.byref(bad)) == 1 and not h.value
    assert opt.dense_product == 0
    for v in (-1, 2):
        lib.glasso_default_options(ctypes.byref(bad))
        bad.dense_product = v
        assert lib.glasso_create(ctypes.byref(h), ctypes.byref(bad)) == 1 and not h.value
    assert lib.glasso_autotune(None, 100, 1, None, None) == 1
    # the covariance rejects a null handle or buffers and empty shapes before any device call
    assert lib.glasso_covariance(None, None, 10, 10, 1, None, None) == 1
    fake = ctypes.c_void_p(1)
    assert lib.glasso_covariance(fake, None, 10, 10, 1, None, None) == 1
    assert lib.glasso_covariance(fake, fake, 0, 10, 1, fake, None) == 1
    assert lib.glasso_covariance(fake, fake, 10, 0, 1, fake, None) == 1
    # the sparse product rejects a null handle or buffer and n < 1 the same way
    assert lib.glasso_sparse_product(None, fake, fake, fake, 10, fake, None, None) == 1
    assert lib.glasso_sparse_product(fake, fake, None, fake, 10, fake, None, None) == 1
    assert lib.glasso_sparse_product(fake, fake, fake, fake, 0, fake, None, None) == 1


def test_struct_layout_matches_c():
    """Compile a probe against the header with gcc and compare sizes/offsets."""
    import paper_2205_10027_amd as g

    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "glasso.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(glasso_options),
         offsetof(glasso_options, warm_start),
         offsetof(glasso_options, tile_policy), offsetof(glasso_options, graphs), offsetof(glasso_options, w_mixed),
         offsetof(glasso_options, ls_width), offsetof(glasso_options, dense_product),
         sizeof(glasso_info), offsetof(glasso_info, nnz), offsetof(glasso_info, status),
         offsetof(glasso_info, time_ms), offsetof(glasso_info, aza_gemm_products),
         offsetof(glasso_info, aza_sparse_products), offsetof(glasso_info, leaf_launches),
         offsetof(glasso_info, leaf_ms), offsetof(glasso_info, leaf_flops), offsetof(glasso_options, screen),
         offsetof(glasso_options, sigma), offsetof(glasso_info, components),
         offsetof(glasso_info, largest_component), offsetof(glasso_options, method));
  return 0;
}'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "probe.c")
        exe = os.path.join(d, "probe")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    want = [ctypes.sizeof(g.GlassoOptions), g.GlassoOptions.warm_start.offset, g.GlassoOptions.tile_policy.offset,
            g.GlassoOptions.graphs.offset, g.GlassoOptions.w_mixed.offset, g.GlassoOptions.ls_width.offset,
            g.GlassoOptions.dense_product.offset, ctypes.sizeof(g.GlassoInfo),
            g.GlassoInfo.nnz.offset, g.GlassoInfo.status.offset, g.GlassoInfo.time_ms.offset,
            g.GlassoInfo.aza_gemm_products.offset, g.GlassoInfo.aza_sparse_products.offset,
            g.GlassoInfo.leaf_launches.offset, g.GlassoInfo.leaf_ms.offset, g.GlassoInfo.leaf_flops.offset,
            g.GlassoOptions.screen.offset, g.GlassoOptions.sigma.offset, g.GlassoInfo.components.offset,
            g.GlassoInfo.largest_component.offset, g.GlassoOptions.method.offset]
    assert [int(x) for x in out] == want
