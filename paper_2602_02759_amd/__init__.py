"""nnef: nonnegative einsum factorization by multiplicative updates on MI355X.

The GPU library is ``libnnef.so`` (C ABI, declared in ``include/nnef.h``);
``paper_2602_02759_amd.nnef`` is its Python binding.  Importing this package
loads nothing; import the submodules you need.
"""
