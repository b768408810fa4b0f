"""mxsten: MI355X-native finite-difference stencils and ADI line solves.

The compute path is the HIP library ``libmxsten.so`` built from ``csrc/``;
``binding`` marshals arguments to its C ABI.
"""
