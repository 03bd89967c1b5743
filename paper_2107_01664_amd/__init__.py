"""tpsurf: the tangent-point hot path of "Repulsive Surfaces" on MI355X (gfx950).

The compute path is the C-ABI library ``libtpsurf.so`` (hand-written HIP kernels);
``paper_2107_01664_amd.tpsurf`` is its thin ctypes binding.  Importing this package
does not load the library; ``meshgen`` builds seeded synthetic inputs.
"""
__all__ = ["meshgen", "tpsurf"]
