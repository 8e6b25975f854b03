"""MI355X-native multigrid solver for the nonlinear f(R) scalar-field equation (ECOSMOG,
arXiv:1110.1379).  The compute path is the HIP library ``libmgfr.so`` built from ``csrc/``;
``mgfr`` is its Python binding (argument marshalling only).  Importing the package loads
nothing; ``paper_1110_1379_amd.mgfr`` loads the library on first use."""
