"""MI355X-native dense-tableau simplex (HIP for gfx950 behind a C ABI).

The binding in `lpdense` loads the in-tree shared library `liblpdense.so`;
it is imported lazily so that `paper_1804_04737_amd.lpgen` (input
generators) can be used without the native library.
"""
__all__ = ["lpdense", "lpgen"]


def __getattr__(name):
    if name in ("lpdense", "lpgen"):
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
