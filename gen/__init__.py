"""Seeded synthetic inputs (reference texts, read batches, request streams)."""
from .workloads import *  # noqa: F401,F403
