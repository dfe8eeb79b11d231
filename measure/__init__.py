"""Measurement tooling of the benchmark (not part of the library): the atomic-throughput probe
the J^T J v kernel's L2 atomic request rate is compared against, and the rocprofv3 profiling
script whose summaries live in profiles/."""
