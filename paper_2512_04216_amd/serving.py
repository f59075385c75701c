"""Serving front end (binding of sv_server_* / sv_submit / sv_poll)."""
from __future__ import annotations


class Server:
    def __init__(self, *a, **k):
        raise NotImplementedError("serving loop not built yet")
