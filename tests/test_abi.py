"""The C-ABI library loads and exports every function include/*.h declares
(no GPU needed: nothing is called)."""
import ctypes
import glob
import os
import re

import paper_1401_6235_amd as tf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w\s\*]*?\b(tf\w*)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return names


def test_header_declares_the_api():
    names = declared_functions()
    for required in ("tf_add", "tf_sub", "tf_mul", "tf_div", "tf_sqrt", "tf_axpy", "tf_horner",
                     "tf_sum", "tf_dot", "tf_coupled", "tf_renorm", "tf_chain", "tf_plain_chain",
                     "tf_trsv_upper", "tf_quadratic", "tf_fma"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = tf.lib()
    missing = [n for n in sorted(declared_functions()) if not hasattr(lib, n)]
    assert not missing, missing


def test_host_only_calls():
    """Calls that touch no device: status strings, version, workspace sizes,
    argument validation that fails before any launch."""
    lib = tf.lib()
    assert lib.tf_strerror(0) == b"success"
    assert lib.tf_version() >= 10000
    assert tf.tf_reduce_workspace_bytes(tf.TF_F64, 0) == 0
    assert tf.tf_reduce_workspace_bytes(tf.TF_F64, 1 << 26) >= (1 << 18) * 16
    # invalid dtype / negative n are rejected before any launch
    assert lib.tf_add(7, ctypes.c_int64(10), None, None, None, None, None, None, None) == -1
    assert lib.tf_add(tf.TF_F64, ctypes.c_int64(-1), None, None, None, None, None, None, None) == -1
    assert lib.tf_horner(tf.TF_F64, ctypes.c_int64(10), 99, None, None, None, None, None, None) == -1
    # n == 0 is a no-op that needs no pointers
    assert lib.tf_mul(tf.TF_F32, ctypes.c_int64(0), None, None, None, None, None, None, None) == 0
    # tuning knobs validate their values
    assert lib.tf_config(tf.TF_CFG_RED_TILES_PER_BLOCK, ctypes.c_int64(3)) == -1
    assert lib.tf_config(tf.TF_CFG_RED_TILES_PER_BLOCK, ctypes.c_int64(512)) == -1
    assert lib.tf_config(tf.TF_CFG_RED_TILES_PER_BLOCK, ctypes.c_int64(-1)) == -1
    assert lib.tf_config(tf.TF_CFG_RED_TILES_PER_BLOCK, ctypes.c_int64(0)) == 0  # default: tuned (0)
    assert lib.tf_config(tf.TF_CFG_RED_WAVES, ctypes.c_int64(2)) == -1
    assert lib.tf_config(tf.TF_CFG_RED_WAVES, ctypes.c_int64(32)) == -1
    assert lib.tf_config(tf.TF_CFG_RED_WAVES, ctypes.c_int64(8)) == 0
    assert lib.tf_config(tf.TF_CFG_RED_WAVES, ctypes.c_int64(0)) == 8
    assert lib.tf_config(99, ctypes.c_int64(1)) == -1
    # the chain, coupled and application calls validate op, mode and sizes
    i64 = ctypes.c_int64
    assert lib.tf_coupled(tf.TF_F64, 5, 0, i64(10), None, None, None, None, None, None, None) == -1
    assert lib.tf_chain(tf.TF_F64, 0, 3, i64(10), i64(1), None, None, None, None, None, None, None) == -1
    assert lib.tf_chain(tf.TF_F64, 0, 0, i64(10), i64(-1), None, None, None, None, None, None, None) == -1
    assert lib.tf_chain(tf.TF_F32, 2, 2, i64(0), i64(5), None, None, None, None, None, None, None) == 0
    assert lib.tf_trsv_upper(tf.TF_F64, i64(4), 0, None, None, None, None, None, None, None) == -1
    assert lib.tf_trsv_upper(tf.TF_F64, i64(4), tf.TF_MAX_TRSV + 1, None, None, None, None, None, None,
                             None) == -1
    assert lib.tf_quadratic(tf.TF_F64, i64(3), *([None] * 10), None) == -1
    assert lib.tf_fma(tf.TF_F32, i64(0), *([None] * 8), None) == 0
    # the allocation-free dot validates its arguments and rejects, on the
    # host and before any device call, partials beyond its static array
    # (2^40 leaves leave 2^24 partials even at 256 tiles per block)
    dummy = ctypes.c_void_p(256)
    assert lib.tf_dot_noalloc(7, i64(10), dummy, None, dummy, None, dummy, None) == -1
    assert lib.tf_dot_noalloc(tf.TF_F64, i64(-1), dummy, None, dummy, None, dummy, None) == -1
    assert lib.tf_dot_noalloc(tf.TF_F64, i64(10), None, None, dummy, None, dummy, None) == -1
    assert lib.tf_dot_noalloc(tf.TF_F64, i64(10), dummy, None, dummy, None, None, None) == -1
    assert lib.tf_dot_noalloc(tf.TF_F64, i64(1 << 40), dummy, None, dummy, None, dummy, None) == -3
    assert lib.tf_dot_noalloc(tf.TF_F32, i64(1 << 40), dummy, None, dummy, None, dummy, None) == -3


def test_c_consumer_builds():
    """The C++ consumer of the ABI (run by the GPU tests) compiles and links
    against the library and the oracle using tf.h alone."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("c_abi_build", os.path.join(ROOT, "tests", "c_abi", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    assert os.path.exists(mod.build())
