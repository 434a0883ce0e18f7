"""MI355X-native X-MeshGraphNet processor hot path.

The compute lives in libxmgn.so (HIP for gfx950, C ABI in include/xmgn.h);
`api` is its thin Python face.  Import `paper_2411_17164_amd.api` to load the
library (it raises ImportError when the library is missing).
"""

__all__ = ["api"]
