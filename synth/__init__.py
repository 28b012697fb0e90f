"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke
check: scheme specifications (step counts and free weights), initial data,
wave-speed fields, source and receiver layouts, and the workload sizes.

This package holds no part of the time-stepping method: it only draws and
shapes inputs.  Both the GPU library's callers and the CPU oracle consume it.
"""
