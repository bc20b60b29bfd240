"""MI355X (gfx950) implementation of the codec of "Fast Compression Method for
Medical Images on the Web" (Hulsken, 2020): colour transform, 5/3 integer
lifting pyramid, quantiser and per-block bitplane / zero-run / Huffman coding,
encode and decode, as HIP kernels behind the C ABI of include/isx.h.

``isx`` is the ctypes binding; ``synth`` draws the seeded synthetic inputs.
"""
