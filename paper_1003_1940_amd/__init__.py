"""MI355X-native bi-directed de Bruijn graph construction (k-mer node table and
canonical bi-directed edge list) by sorting, after Kundeti et al.

The HIP library ``libdbg.so`` does all the work; ``api`` marshals arguments.
"""
from . import api  # noqa: F401
from .api import build, build_async, pack, workspace_bytes, Workspace, Graph, DbgError  # noqa: F401
