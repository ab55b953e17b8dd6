"""Convenience wrapper around the streaming entry points of the C ABI."""

import numpy as np

from . import _lib


class TRStream:
    """Owns one ``tr_stream`` handle.

    X_init and batches are (I_1, .., I_{N-1}, t) arrays (NumPy on the host, or
    torch tensors on the device); cores are (R_n, I_n, R_{n+1}) arrays with the
    temporal core holding t_init slices.  With cores_init None the library
    initialises the cores by batch TR-ALS on X_init (``ranks`` required).
    """

    def __init__(self, X_init, cores_init=None, compute_dtype="f64", sketch=None,
                 sketch_size=0, rescale=True, temporal_literal=True, seed=0, max_slices=0,
                 check_finite=False, device=0, hip_stream=None, ranks=None, sweeps=1,
                 init_max_sweeps=0, init_tol=0.0):
        self.dims = list(X_init.shape[:-1])
        if cores_init is not None:
            self.ranks = [int(G.shape[0]) for G in cores_init]
        else:
            self.ranks = [int(r) for r in ranks]
        self.N = len(self.ranks)
        self.handle = _lib.tr_stream_init(
            X_init, cores_init, self.ranks, compute_dtype=compute_dtype, sketch=sketch,
            sketch_size=sketch_size, rescale=rescale, temporal_literal=temporal_literal,
            seed=seed, max_slices=max_slices, check_finite=check_finite, device=device,
            hip_stream=hip_stream, sweeps=sweeps, init_max_sweeps=init_max_sweeps,
            init_tol=init_tol)
        self.sketch_size = int(sketch_size)
        self._keep = None

    @classmethod
    def load(cls, path, dims, ranks, compute_dtype="f64", sketch=None, sketch_size=0,
             device=0, hip_stream=None, max_slices=0):
        """A stream resumed from a file written by ``save``; the shape and
        options given must be the saved ones (the library checks them)."""
        self = cls.__new__(cls)
        self.handle = None
        self.dims = [int(i) for i in dims]
        self.ranks = [int(r) for r in ranks]
        self.N = len(self.ranks)
        self.sketch_size = int(sketch_size)
        self._keep = None
        self.handle = _lib.tr_stream_load(path, dims=self.dims, ranks=self.ranks,
                                          compute_dtype=compute_dtype, sketch=sketch,
                                          sketch_size=sketch_size, device=device,
                                          hip_stream=hip_stream, max_slices=max_slices)
        return self

    def save(self, path):
        _lib.tr_stream_save(self.handle, path)

    def set_samples(self, idxs=None, signs=None):
        _lib.tr_stream_set_samples(self.handle, idxs, signs)

    def stats(self):
        return _lib.tr_stream_get_stats(self.handle)

    def d(self, n):
        return self.ranks[n] * self.ranks[(n + 1) % self.N]

    def update(self, X_new):
        self._keep = _lib.tr_stream_update(self.handle, X_new)

    def samples(self):
        return _lib.tr_stream_get_samples(self.handle, self.N, self.sketch_size)

    def sync(self):
        _lib.tr_stream_sync(self.handle)

    def profile(self, enable=True):
        _lib.tr_stream_profile(self.handle, enable)

    def profile_read(self, kind):
        return _lib.tr_stream_profile_read(self.handle, kind)

    def num_slices(self):
        return _lib.tr_stream_num_slices(self.handle)

    def reconstruct_error(self, X_all):
        return _lib.tr_reconstruct_error(self.handle, X_all)

    def cores(self):
        return _lib.tr_stream_get_cores(self.handle, self.dims, self.ranks)

    def PQ(self, n):
        return _lib.tr_stream_get_PQ(self.handle, n, self.dims[n], self.d(n))

    def close(self):
        if self.handle:
            _lib.tr_stream_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
