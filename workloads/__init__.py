"""Seeded synthetic inputs (files and access lists) shared by the oracle and the GPU path.

Holds none of the page-cache method's arithmetic.
"""
