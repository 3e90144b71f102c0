"""MI355X-native projected tensor-tensor product *_Q and truncated tSVDQ
(Keegan & Newman, arXiv:2409.19402) on hand-written gfx950 HIP kernels.

`binding` holds the Python entry points (qprod, proj, tsvdq, hat, unhat,
facewise, their adjoints, check_q); they call the C ABI declared in
include/projprod.h.  `synth` builds seeded synthetic inputs.
"""

__version__ = "0.1.0"


def __getattr__(name):
    # the binding needs torch; import it on first use so `synth` stays light
    if name in ("binding",):
        import importlib
        return importlib.import_module(f"{__name__}.binding")
    raise AttributeError(name)
