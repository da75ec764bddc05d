"""MI355X (gfx950) implementation of the per-event ML tracking chain of
arXiv:2501.05520 Section 2.2.2 behind the C ABI of include/trk.h.  The compute
lives in libtrk.so (HIP); `trk` is its ctypes binding."""
