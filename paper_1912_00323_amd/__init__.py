"""Exact hypercube-grid DBSCAN (HCA-DBSCAN, arXiv 1912.00323) on AMD MI355X.

The compute path is the HIP library ``libhca.so`` behind the C ABI declared in
``include/hca.h``; :mod:`paper_1912_00323_amd.hca` is its thin Python binding.
Importing this package loads nothing; the library is loaded on first use.
"""
__all__ = ["hca", "datagen"]
