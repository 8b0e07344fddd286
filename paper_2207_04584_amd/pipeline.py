"""Many fields gridded one at a time through a first-in-first-out queue
served by host threads, each with a stream of its own: a field's setup and
then its channel kernel run on the stream of the thread that took it.  This
is the shape of the paper's multi-stream pipeline for many small fields
(Sec. 4.2: fields handed in turn to CPU workers, each driving GPU streams),
kept beside the batched form (hg_batch_*: every field's setup, then one
graph-held launch over all of them) so the two can be timed on the same
fields.  The arithmetic is the library's; this module only schedules calls.
"""
import queue
import threading

from . import api


def grid_fields_fifo(fields, n_streams=4, precision=api.HG_PREC_FP32, chunk=0):
    """fields: dicts with "ra", "dec" (host or device FP64), "map", "kernel"
    and "values" (a device tensor [n][C], or None for no channels), as for
    api.Batch.  Returns the float32 device maps [C][ny][nx] in field order
    (None where a field has no channels).  Plans stay open until every field
    is done, so that no worker waits on another's work while freeing its
    plan; they are closed before returning."""
    torch = api._torch()
    api.lib()  # loaded once, before any worker calls into it
    outs = []
    for f in fields:
        v = f.get("values")
        if v is None:
            outs.append(None)
        else:
            ny, nx = int(f["map"]["ny"]), int(f["map"]["nx"])
            outs.append(torch.empty((v.shape[1], ny, nx), dtype=torch.float32, device=v.device))
    torch.cuda.synchronize()
    todo = queue.Queue()
    for i in range(len(fields)):
        todo.put(i)
    plans = [None] * len(fields)
    errors = []

    def worker():
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            while not errors:
                try:
                    i = todo.get_nowait()
                except queue.Empty:
                    break
                f = fields[i]
                try:
                    # chunk lengths as a batch's fields take them (predicted
                    # from the support), so the two forms give the same maps
                    p = api.Plan(f["ra"], f["dec"], f["map"], f["kernel"], precision=precision,
                                 chunk=chunk, predict_chunk=True, stream=s)
                    plans[i] = p
                    if f.get("values") is not None:
                        p.grid(f["values"], out=outs[i], stream=s)
                except Exception as e:  # reported after every worker has stopped
                    errors.append((i, e))
        s.synchronize()

    threads = [threading.Thread(target=worker) for _ in range(max(1, min(n_streams, len(fields))))]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    torch.cuda.synchronize()
    for p in plans:
        if p is not None:
            p.close()
    if errors:
        i, e = min(errors, key=lambda x: x[0])
        raise api.HegridError(getattr(e, "status", api.HG_ERR_INTERNAL), f"field {i}: {e}")
    return outs
