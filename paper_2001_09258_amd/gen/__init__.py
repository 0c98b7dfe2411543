"""Build-time generators for the kernels' constant data (polynomial
coefficients and the Payne-Hanek table).  They run on the host with mpmath
and write checked-in ``csrc/generated/*.inc`` headers; nothing here runs when
the library is used."""
