"""MI355X (gfx950) implementation of the PBM + multigrid-MINRES hot path for
the 3D variable thickness sheet problem (Brune & Kocvara, arXiv 1904.06556).

    paper_1904_06556_amd.vts      ctypes binding of libvts (include/vts.h)
    paper_1904_06556_amd.build    builds libvts.so with hipcc for gfx950
"""
__all__ = ["vts", "build"]
