"""Oracle: a plain, slow, fp64 CPU implementation of Universal Beta Splatting.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, links or
runs anything here; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path: it parses the parameter format itself, evaluates every step in float64
in the paper's order and notation, and gets its gradients from torch's fp64
autograd (per-primitive steps) and a hand-written per-pixel adjoint in plain
C (compositing), never from the GPU kernels.

Modules
-------
``preprocess``  per-primitive steps (Section 4 of the paper): parameter
                activation, spatial-orthogonal Cholesky covariance,
                query, Beta-modulated opacity and conditioning, pinhole
                projection to a screen-space record.
``raster``      per-pixel compositing without tiles (Section 3 compositing
                equation with the Beta kernel of Section 3/4.3), its adjoint,
                and the binning reference (exact ellipse/tile test, keys,
                stable sort, per-tile ranges).
``render``      end-to-end render and gradients for a scene and views.
"""
